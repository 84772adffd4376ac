/* links_ref.c -- FP64 CPU oracle (test infrastructure only; see links_ref.h).
 *
 * Plain, slow, single-candidate-at-a-time code written to be checked by eye
 * against the paper:
 *   - representation: adjacency matrix plus per-joint type and initial position;
 *     link lengths come from the initial positions (Methodology, "Mechanism
 *     Representation"); joints 0 and 1 form the actuator arm by default
 *     (Methodology, "Dataset Features & Statistics", item 1).
 *   - solve order: starting from the fixed joints and the actuated joint, every
 *     joint with two known neighbours is solved, round after round, until all are
 *     known; complex loops leave joints unsolved (Methodology, "Graphical
 *     Simulator").
 *   - simulation: the actuator arm turns through T equally spaced positions of a
 *     full rotation (Methodology, "Dataset Features & Statistics", item 2; T = 200
 *     there, 50 for the low-fidelity pass of "Scale of Infeasibilities"); a
 *     mechanism is valid when the full rotation completes without locking
 *     (Methodology, "Finding Valid Initial Positions").
 *   - each joint is placed from its two known parents by the textbook
 *     circle-circle intersection (the paper does not print the formula) and the
 *     branch is the intersection nearer the joint's previous position; a variant
 *     keeps every joint on the side of its parents' line where it starts (the
 *     paper leaves the rule open: it takes the initial positions into account and
 *     evaluates the actuator positions independently).
 *   - path normalisation (Methodology, "Dataset Curation & Processing"): the
 *     diameter rule, plus a centroid / RMS / principal-axis variant.
 *
 * Compiled with -O2 -ffp-contract=off and no fast-math so every operation is a
 * single IEEE-754 double operation in the order written.
 */
#include "links_ref.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define MAXJ 32

static int popcount32(uint32_t x) {
  int c = 0;
  while (x) {
    x &= x - 1u;
    c++;
  }
  return c;
}

static int lowest_bit(uint32_t x) {
  for (int i = 0; i < 32; i++)
    if ((x >> i) & 1u) return i;
  return -1;
}

static uint32_t low_mask(int n) { return n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u); }

/* Integer structure of one candidate: symmetric adjacency with empty diagonal and
 * nothing beyond joint n-1; pivot fixed, tip free, and the actuator arm present. */
static int structure_ok(int J, int n, const uint32_t* adj, uint32_t fixed, int pivot, int tip) {
  if (n < 3 || n > J) return 0;
  uint32_t live = low_mask(n);
  if (fixed & ~live) return 0;
  for (int i = 0; i < J; i++) {
    if (i >= n) {
      if (adj[i] != 0u) return 0;
      continue;
    }
    if (adj[i] & ~live) return 0;
    if ((adj[i] >> i) & 1u) return 0;
    for (int j = 0; j < n; j++)
      if (((adj[i] >> j) & 1u) != ((adj[j] >> i) & 1u)) return 0;
  }
  if (pivot >= n || tip >= n || pivot == tip) return 0;
  if (!((fixed >> pivot) & 1u)) return 0;
  if ((fixed >> tip) & 1u) return 0;
  if (!((adj[pivot] >> tip) & 1u)) return 0;
  return 1;
}

/* Rounds of the graphical solver.  Round r solves, in ascending joint index, every
 * unknown joint with at least two known neighbours; its parents are the two
 * smallest known neighbours.  Returns 1 when every joint ends up known. */
static int solve_order_one(int n, const uint32_t* adj, uint32_t fixed, int tip, int8_t* order,
                           int* n_dyads, int* depth) {
  uint32_t known = fixed | (1u << tip);
  int nd = 0;
  int rounds = 0;
  for (;;) {
    uint32_t solved_now = 0u;
    for (int k = 0; k < n; k++) {
      if ((known >> k) & 1u) continue;
      uint32_t kn = adj[k] & known;
      if (popcount32(kn) < 2) continue;
      int a = lowest_bit(kn);
      int b = lowest_bit(kn & ~(1u << a));
      order[3 * nd + 0] = (int8_t)k;
      order[3 * nd + 1] = (int8_t)a;
      order[3 * nd + 2] = (int8_t)b;
      nd++;
      solved_now |= 1u << k;
    }
    if (solved_now == 0u) break;
    known |= solved_now;
    rounds++;
  }
  *n_dyads = nd;
  *depth = rounds;
  return known == low_mask(n);
}

int links_ref_solve_order(int32_t B, int32_t J, const uint8_t* n, const uint32_t* adj,
                          const uint32_t* fixed, const uint8_t* motor, int8_t* order,
                          uint8_t* n_dyads, uint8_t* depth, uint8_t* status) {
  if (B < 0 || J < 1 || J > MAXJ) return -1;
  if (B > 0 && (!n || !adj || !fixed || !motor || !order || !n_dyads || !depth || !status)) return -1;
  for (int32_t c = 0; c < B; c++) {
    int8_t* ord = order + (size_t)c * J * 3;
    for (int i = 0; i < J * 3; i++) ord[i] = -1;
    n_dyads[c] = 0;
    depth[c] = 0;
    const uint32_t* A = adj + (size_t)c * J;
    int pivot = motor[2 * c], tip = motor[2 * c + 1];
    if (!structure_ok(J, n[c], A, fixed[c], pivot, tip)) {
      status[c] = LREF_BAD_MECH;
      continue;
    }
    int nd = 0, dp = 0;
    int complete = solve_order_one(n[c], A, fixed[c], tip, ord, &nd, &dp);
    n_dyads[c] = (uint8_t)nd;
    depth[c] = (uint8_t)dp;
    status[c] = complete ? LREF_VALID : LREF_UNSOLVABLE;
  }
  return 0;
}

/* ------------------------------------------------------------------ simulation */

typedef struct {
  int32_t B, J, T, out_joint;
  const uint8_t* n;
  const uint32_t* adj;
  const uint32_t* fixed;
  const uint8_t* motor;
  const double* x0;
  double tau_drift;
  uint8_t* status;
  int16_t* fail_step;
  double* path;
  double* pos_all;
  double* margins;
  int32_t branch; /* LREF_BRANCH_CONTINUITY or LREF_BRANCH_ORIENTATION */
} sim_args;

static double sq_dist(const double* p, const double* q) {
  double dx = p[0] - q[0];
  double dy = p[1] - q[1];
  return dx * dx + dy * dy;
}

static void simulate_one(const sim_args* A, int32_t c) {
  const int J = A->J, T = A->T;
  const int n = A->n[c];
  const uint32_t* adj = A->adj + (size_t)c * J;
  const uint32_t fixed = A->fixed[c];
  const int pivot = A->motor[2 * c], tip = A->motor[2 * c + 1];
  const double* x0 = A->x0 + (size_t)c * J * 2;
  double* path = A->path ? A->path + (size_t)c * T * 2 : NULL;
  double* all = A->pos_all ? A->pos_all + (size_t)c * T * J * 2 : NULL;
  double m_disc = INFINITY, m_deg = INFINITY, m_branch = INFINITY, m_drift = INFINITY;

  if (path)
    for (int i = 0; i < T * 2; i++) path[i] = NAN;
  if (all)
    for (size_t i = 0; i < (size_t)T * J * 2; i++) all[i] = NAN;
  A->fail_step[c] = -1;

  /* validation: integer structure, finite positions and non-zero link lengths */
  int ok = structure_ok(J, n, adj, fixed, pivot, tip);
  if (ok) {
    for (int i = 0; i < n; i++)
      if (!isfinite(x0[2 * i]) || !isfinite(x0[2 * i + 1])) ok = 0;
  }
  double scale = 0.0;
  if (ok) {
    for (int i = 0; i < n; i++)
      for (int j = i + 1; j < n; j++)
        if ((adj[i] >> j) & 1u) {
          double L = sqrt(sq_dist(x0 + 2 * i, x0 + 2 * j));
          if (!(L > 1e-12)) ok = 0;
          if (L > scale) scale = L;
        }
  }
  if (!ok) {
    A->status[c] = LREF_BAD_MECH;
    goto done;
  }

  int8_t order[MAXJ * 3];
  int nd = 0, dp = 0;
  if (!solve_order_one(n, adj, fixed, tip, order, &nd, &dp)) {
    A->status[c] = LREF_UNSOLVABLE;
    goto done;
  }

  /* edges used by the solve: the actuator arm and every (joint, parent) pair;
   * every other link is redundant and is checked for length drift */
  uint32_t used[MAXJ];
  memset(used, 0, sizeof(used));
  used[pivot] |= 1u << tip;
  used[tip] |= 1u << pivot;
  for (int s = 0; s < nd; s++) {
    int k = order[3 * s], a = order[3 * s + 1], b = order[3 * s + 2];
    used[k] |= (1u << a) | (1u << b);
    used[a] |= 1u << k;
    used[b] |= 1u << k;
  }

  int out = A->out_joint;
  if (out < 0) out = nd > 0 ? order[3 * (nd - 1)] : tip;

  const double scale2 = scale * scale;
  const double deg_thr = 1e-12 * scale2;
  const double vx = x0[2 * tip] - x0[2 * pivot];
  const double vy = x0[2 * tip + 1] - x0[2 * pivot + 1];

  double pos[MAXJ][2], prev[MAXJ][2];
  for (int i = 0; i < n; i++) {
    prev[i][0] = x0[2 * i];
    prev[i][1] = x0[2 * i + 1];
  }
  /* orientation rule: the side of a->b on which each placed joint starts
   * (z of (x0_b - x0_a) x (x0_k - x0_a) >= 0: left, ties left) */
  int left0[MAXJ];
  for (int s = 0; s < nd; s++) {
    int k = order[3 * s], a = order[3 * s + 1], b = order[3 * s + 2];
    double cr = (x0[2 * b] - x0[2 * a]) * (x0[2 * k + 1] - x0[2 * a + 1]) -
                (x0[2 * b + 1] - x0[2 * a + 1]) * (x0[2 * k] - x0[2 * a]);
    left0[s] = cr >= 0.0;
  }

  for (int t = 0; t < T; t++) {
    /* actuator: fixed joints stay at x0, the tip turns by theta_t about the pivot */
    double theta = 2.0 * M_PI * (double)t / (double)T;
    double ct = cos(theta), st = sin(theta);
    for (int i = 0; i < n; i++)
      if ((fixed >> i) & 1u) {
        pos[i][0] = x0[2 * i];
        pos[i][1] = x0[2 * i + 1];
      }
    pos[tip][0] = x0[2 * pivot] + (ct * vx - st * vy);
    pos[tip][1] = x0[2 * pivot + 1] + (st * vx + ct * vy);

    /* dyads in solve order: circle about parent a of radius |x0_k - x0_a| meets
     * circle about parent b of radius |x0_k - x0_b| */
    int fail = LREF_VALID;
    for (int s = 0; s < nd && fail == LREF_VALID; s++) {
      int k = order[3 * s], a = order[3 * s + 1], b = order[3 * s + 2];
      double ra2 = sq_dist(x0 + 2 * k, x0 + 2 * a);
      double rb2 = sq_dist(x0 + 2 * k, x0 + 2 * b);
      double ra = sqrt(ra2), rb = sqrt(rb2);
      double dx = pos[b][0] - pos[a][0];
      double dy = pos[b][1] - pos[a][1];
      double d2 = dx * dx + dy * dy;
      if (d2 / scale2 < m_deg) m_deg = d2 / scale2;
      if (d2 <= deg_thr) {
        fail = LREF_DEGENERATE;
        break;
      }
      /* discriminant of the circle-circle intersection,
       * K = 4 d^2 ra^2 - (d^2 + ra^2 - rb^2)^2 = 16 area(a,b,k)^2 (Heron);
       * the circles miss each other (the mechanism locks) when K < 0 */
      double sum = ra + rb, dif = ra - rb;
      double K = (sum * sum - d2) * (d2 - dif * dif);
      double disc = K / (4.0 * scale2); /* units of length^2; h^2 (d/scale)^2 */
      if (fabs(disc) / scale2 < m_disc) m_disc = fabs(disc) / scale2;
      if (K < 0.0) {
        fail = LREF_LOCKED;
        break;
      }
      double d = sqrt(d2);
      double h = sqrt(K) / (2.0 * d);              /* height of k over the base a-b */
      double along = (d2 + ra2 - rb2) / (2.0 * d); /* foot of that height, from a */
      double bx = pos[a][0] + (along / d) * dx;
      double by = pos[a][1] + (along / d) * dy;
      double ox = -(h / d) * dy;
      double oy = (h / d) * dx;
      double cpx = bx + ox, cpy = by + oy; /* left of a->b */
      double cmx = bx - ox, cmy = by - oy; /* right of a->b */
      /* branch: the intersection nearer the previous position (tie: left), or
       * the starting side of a->b */
      int left;
      if (A->branch == LREF_BRANCH_ORIENTATION) {
        left = left0[s];
      } else {
        double dp2 = (prev[k][0] - cpx) * (prev[k][0] - cpx) + (prev[k][1] - cpy) * (prev[k][1] - cpy);
        double dm2 = (prev[k][0] - cmx) * (prev[k][0] - cmx) + (prev[k][1] - cmy) * (prev[k][1] - cmy);
        double side = fabs((prev[k][0] - bx) * (-dy) + (prev[k][1] - by) * dx) / d;
        if (side / scale < m_branch) m_branch = side / scale;
        left = dp2 <= dm2;
      }
      if (left) {
        pos[k][0] = cpx;
        pos[k][1] = cpy;
      } else {
        pos[k][0] = cmx;
        pos[k][1] = cmy;
      }
    }

    /* redundant links must keep their initial length */
    if (fail == LREF_VALID) {
      for (int i = 0; i < n && fail == LREF_VALID; i++)
        for (int j = i + 1; j < n; j++) {
          if (!((adj[i] >> j) & 1u) || ((used[i] >> j) & 1u)) continue;
          double L = sqrt(sq_dist(x0 + 2 * i, x0 + 2 * j));
          double now = sqrt(sq_dist(pos[i], pos[j]));
          double drift = fabs(now - L);
          double md = fabs(drift - A->tau_drift * scale) / scale;
          if (md < m_drift) m_drift = md;
          if (drift > A->tau_drift * scale) {
            fail = LREF_DRIFT;
            break;
          }
        }
    }

    if (fail != LREF_VALID) {
      A->status[c] = (uint8_t)fail;
      A->fail_step[c] = (int16_t)t;
      goto done;
    }
    if (path && out < n) {
      path[2 * t] = pos[out][0];
      path[2 * t + 1] = pos[out][1];
    }
    if (all)
      for (int i = 0; i < n; i++) {
        all[((size_t)t * J + i) * 2] = pos[i][0];
        all[((size_t)t * J + i) * 2 + 1] = pos[i][1];
      }
    for (int i = 0; i < n; i++) {
      prev[i][0] = pos[i][0];
      prev[i][1] = pos[i][1];
    }
  }
  A->status[c] = LREF_VALID;

done:
  if (A->margins) {
    double* m = A->margins + (size_t)c * 4;
    m[0] = m_disc;
    m[1] = m_deg;
    m[2] = m_branch;
    m[3] = m_drift;
  }
}

typedef struct {
  const sim_args* args;
  int32_t lo, hi;
} sim_chunk;

static void* sim_worker(void* p) {
  sim_chunk* ch = (sim_chunk*)p;
  for (int32_t c = ch->lo; c < ch->hi; c++) simulate_one(ch->args, c);
  return NULL;
}

int links_ref_simulate(int32_t B, int32_t J, const uint8_t* n, const uint32_t* adj,
                       const uint32_t* fixed, const uint8_t* motor, const double* x0,
                       int32_t T, int32_t out_joint, double tau_drift, uint8_t* status,
                       int16_t* fail_step, double* path,
                       double* pos_all, double* margins, int32_t nthreads) {
  return links_ref_simulate_branch(B, J, n, adj, fixed, motor, x0, T, out_joint, tau_drift, status, fail_step,
                                   path, pos_all, margins, nthreads, LREF_BRANCH_CONTINUITY);
}

int links_ref_simulate_branch(int32_t B, int32_t J, const uint8_t* n, const uint32_t* adj,
                              const uint32_t* fixed, const uint8_t* motor, const double* x0,
                              int32_t T, int32_t out_joint, double tau_drift, uint8_t* status,
                              int16_t* fail_step, double* path,
                              double* pos_all, double* margins, int32_t nthreads, int32_t branch) {
  if (B < 0 || J < 1 || J > MAXJ || T < 1 || out_joint >= J) return -1;
  if (branch != LREF_BRANCH_CONTINUITY && branch != LREF_BRANCH_ORIENTATION) return -1;
  if (B > 0 && (!n || !adj || !fixed || !motor || !x0 || !status || !fail_step)) return -1;
  sim_args args = {B, J, T, out_joint, n, adj, fixed, motor, x0, tau_drift,
                   status, fail_step, path, pos_all, margins, branch};
  if (nthreads <= 1 || B < 2) {
    for (int32_t c = 0; c < B; c++) simulate_one(&args, c);
    return 0;
  }
  if (nthreads > B) nthreads = B;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
  sim_chunk* ch = (sim_chunk*)malloc(sizeof(sim_chunk) * (size_t)nthreads);
  if (!th || !ch) {
    free(th);
    free(ch);
    for (int32_t c = 0; c < B; c++) simulate_one(&args, c);
    return 0;
  }
  char* joined = (char*)calloc((size_t)nthreads, 1);
  for (int i = 0; i < nthreads; i++) {
    ch[i].args = &args;
    ch[i].lo = (int32_t)((int64_t)B * i / nthreads);
    ch[i].hi = (int32_t)((int64_t)B * (i + 1) / nthreads);
    if (pthread_create(&th[i], NULL, sim_worker, &ch[i]) != 0) {
      sim_worker(&ch[i]); /* could not start a thread: run the chunk here */
      if (joined) joined[i] = 1;
    }
  }
  for (int i = 0; i < nthreads; i++)
    if (!joined || !joined[i]) pthread_join(th[i], NULL);
  free(joined);
  free(th);
  free(ch);
  return 0;
}

/* ------------------------------------------------------------------ normalisation */

static void rotate(double c, double s, double x, double y, double* ox, double* oy) {
  /* rotation by -phi with c = cos(phi), s = sin(phi) */
  *ox = c * x + s * y;
  *oy = -s * x + c * y;
}

static void normalize_pca(const double* p, int T, double* out, double* xf) {
  double cx = 0.0, cy = 0.0;
  for (int t = 0; t < T; t++) {
    cx += p[2 * t];
    cy += p[2 * t + 1];
  }
  cx /= T;
  cy /= T;
  double ms = 0.0;
  for (int t = 0; t < T; t++) {
    double qx = p[2 * t] - cx, qy = p[2 * t + 1] - cy;
    ms += qx * qx + qy * qy;
  }
  double s = sqrt(ms / T);
  int flags = 0;
  if (!(s >= 1e-12)) {
    for (int t = 0; t < 2 * T; t++) out[t] = 0.0;
    xf[0] = cx;
    xf[1] = cy;
    xf[2] = 0.0;
    xf[3] = 0.0;
    xf[4] = LREF_NF_CONSTANT;
    return;
  }
  double cxx = 0.0, cxy = 0.0, cyy = 0.0;
  for (int t = 0; t < T; t++) {
    double qx = (p[2 * t] - cx) / s, qy = (p[2 * t + 1] - cy) / s;
    cxx += qx * qx;
    cxy += qx * qy;
    cyy += qy * qy;
  }
  cxx /= T;
  cxy /= T;
  cyy /= T;
  /* principal axis of the population covariance */
  double gap = sqrt((cxx - cyy) * (cxx - cyy) + 4.0 * cxy * cxy); /* lambda1 - lambda2 */
  double phi = 0.5 * atan2(2.0 * cxy, cxx - cyy);
  if (gap < 1e-4 * (cxx + cyy)) {
    phi = 0.0;
    flags |= LREF_NF_ISOTROPIC;
  }
  double c = cos(phi), sn = sin(phi);
  double m3 = 0.0;
  for (int t = 0; t < T; t++) {
    double qx = (p[2 * t] - cx) / s, qy = (p[2 * t + 1] - cy) / s;
    double rx, ry;
    rotate(c, sn, qx, qy, &rx, &ry);
    out[2 * t] = rx;
    out[2 * t + 1] = ry;
    m3 += rx * rx * rx;
  }
  /* sign of the principal axis: the third moment along +x is non-negative */
  if (fabs(m3) < 1e-6 * T) {
    flags |= LREF_NF_SIGN_TIE;
  } else if (m3 < 0.0) {
    phi += M_PI;
    for (int t = 0; t < 2 * T; t++) out[t] = -out[t];
  }
  xf[0] = cx;
  xf[1] = cy;
  xf[2] = s;
  xf[3] = phi;
  xf[4] = flags;
}

static void normalize_diameter(const double* p, int T, double* out, double* xf) {
  /* line of maximum distance: first pair (i<j) in lexicographic order */
  int bi = 0, bj = 0;
  double best = -1.0;
  for (int i = 0; i < T; i++)
    for (int j = i + 1; j < T; j++) {
      double d2 = sq_dist(p + 2 * i, p + 2 * j);
      if (d2 > best) {
        best = d2;
        bi = i;
        bj = j;
      }
    }
  int flags = 0;
  if (!(best > 0.0) || !(sqrt(best) >= 1e-12)) {
    for (int t = 0; t < 2 * T; t++) out[t] = 0.0;
    xf[0] = p[0];
    xf[1] = p[1];
    xf[2] = 0.0;
    xf[3] = 0.0;
    xf[4] = LREF_NF_CONSTANT;
    return;
  }
  for (int i = 0; i < T; i++)
    for (int j = i + 1; j < T; j++) {
      if (i == bi && j == bj) continue;
      if (sq_dist(p + 2 * i, p + 2 * j) >= (1.0 - 1e-6) * best) flags |= LREF_NF_DIAM_TIE;
    }
  double D = sqrt(best);
  double ux = p[2 * bj] - p[2 * bi], uy = p[2 * bj + 1] - p[2 * bi + 1];
  double phi = atan2(uy, ux);
  double c = cos(phi), sn = sin(phi);
  /* rotate the diameter to +x, scale it to 1, then centre the bounding box at (0.5,0.5) */
  double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
  for (int t = 0; t < T; t++) {
    double rx, ry;
    rotate(c, sn, p[2 * t] - p[2 * bi], p[2 * t + 1] - p[2 * bi + 1], &rx, &ry);
    rx /= D;
    ry /= D;
    out[2 * t] = rx;
    out[2 * t + 1] = ry;
    if (rx < xmin) xmin = rx;
    if (rx > xmax) xmax = rx;
    if (ry < ymin) ymin = ry;
    if (ry > ymax) ymax = ry;
  }
  double mx = 0.5 * (xmin + xmax), my = 0.5 * (ymin + ymax);
  for (int t = 0; t < T; t++) {
    out[2 * t] = out[2 * t] - mx + 0.5;
    out[2 * t + 1] = out[2 * t + 1] - my + 0.5;
  }
  /* centre in the input frame: p_bi + D * R(phi) (mx, my) */
  xf[0] = p[2 * bi] + D * (c * mx - sn * my);
  xf[1] = p[2 * bi + 1] + D * (sn * mx + c * my);
  xf[2] = D;
  xf[3] = phi;
  xf[4] = flags;
}

int links_ref_normalize_paths(const double* paths, int32_t P, int32_t T, int32_t mode,
                              double* out, double* xform) {
  if (P < 0 || T < 1 || (mode != LREF_NORM_PCA && mode != LREF_NORM_DIAMETER)) return -1;
  if (P > 0 && (!paths || !out || !xform)) return -1;
  for (int32_t i = 0; i < P; i++) {
    const double* p = paths + (size_t)i * T * 2;
    double* o = out + (size_t)i * T * 2;
    double* xf = xform + (size_t)i * 5;
    if (mode == LREF_NORM_PCA)
      normalize_pca(p, T, o, xf);
    else
      normalize_diameter(p, T, o, xf);
  }
  return 0;
}

/* Curation (Methodology, "Dataset Curation & Processing"): arcs are recognised
 * from the mechanism (the path's joint is linked to a ground joint), circles from
 * the normalised path (small variance of the distances from the centre of the
 * unit box), and a mechanism is reduced to the joints the path's joint depends on
 * through the solve order. */
int links_ref_curate(int32_t J, const uint8_t* n, const uint32_t* adj, const uint32_t* fixed,
                     const uint8_t* motor, int32_t out_joint, const int32_t* cand, int32_t P,
                     const double* norm, int32_t T, double circle_var, uint8_t* flags, double* radial_var,
                     uint32_t* keep) {
  if (P < 0 || T < 1 || J < 1 || J > MAXJ) return -1;
  if (P > 0 && (!n || !adj || !fixed || !motor || !norm || !flags || !radial_var || !keep)) return -1;
  for (int32_t i = 0; i < P; i++) {
    const int32_t c = cand ? cand[i] : i;
    const uint32_t* a = adj + (size_t)c * J;
    const int pivot = motor[2 * c], tip = motor[2 * c + 1];
    int8_t order[MAXJ * 3];
    int nd = 0, dp = 0;
    flags[i] = 0;
    keep[i] = 0u;
    /* radial variance of the normalised path about (0.5, 0.5), two passes */
    const double* q = norm + (size_t)i * T * 2;
    double mean = 0.0;
    for (int t = 0; t < T; t++) {
      double dx = q[2 * t] - 0.5, dy = q[2 * t + 1] - 0.5;
      mean += sqrt(dx * dx + dy * dy);
    }
    mean /= (double)T;
    double var = 0.0;
    for (int t = 0; t < T; t++) {
      double dx = q[2 * t] - 0.5, dy = q[2 * t + 1] - 0.5;
      double e = sqrt(dx * dx + dy * dy) - mean;
      var += e * e;
    }
    var /= (double)T;
    radial_var[i] = var;
    /* only a well-formed mechanism that the solver can place is curated */
    if (!structure_ok(J, n[c], a, fixed[c], pivot, tip)) continue;
    if (!solve_order_one(n[c], a, fixed[c], tip, order, &nd, &dp)) continue;
    int out = out_joint >= 0 ? out_joint : (nd > 0 ? order[3 * (nd - 1)] : tip);
    uint32_t f = 0u;
    if (a[out] & fixed[c]) f |= LREF_CUR_ARC;
    if (var < circle_var) f |= LREF_CUR_CIRCLE;
    flags[i] = (uint8_t)f;
    /* ancestors of the path's joint, walking the solve order backwards */
    uint32_t m = 1u << out;
    for (int s = nd - 1; s >= 0; s--) {
      int k = order[3 * s];
      if ((m >> k) & 1u) m |= (1u << order[3 * s + 1]) | (1u << order[3 * s + 2]);
    }
    if ((m >> tip) & 1u) m |= 1u << pivot;
    keep[i] = m;
  }
  return 0;
}
