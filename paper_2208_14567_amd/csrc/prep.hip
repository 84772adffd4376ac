// prep.hip -- once-per-mechanism work: validation, graphical solve order, the LDS
// slot layout used by the simulation kernels and the per-candidate constants;
// plus the small scheduling kernels (bucket sort by solve-order length, valid-path
// compaction, fills).
//
// The solve order follows the paper's graphical solver (Methodology, "Graphical
// Simulator"): starting from the fixed joints and the actuated tip, each round
// places every unknown joint that has two known neighbours; the order is found
// once per mechanism and reused for every actuator position.
#include "common.h"
#include "kernels.h"

namespace links {

namespace {

__device__ inline int popc(uint32_t x) { return __popc(x); }
__device__ inline int lowbit(uint32_t x) { return __ffs(x) - 1; }
__device__ inline uint32_t live_mask(int n) { return n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u); }

constexpr int kPrepBlock = 128;   // solve-order kernel
constexpr int kSortBlock = 64;    // count and fill kernels: one wave, rows staged in LDS

// A candidate's adjacency rows and initial positions, read in place from global
// memory (Global) or from the workgroup's LDS copy with the lanes interleaved
// (Staged: element i of lane l at [i][l]).
struct GlobalRow {
  const uint32_t* adj;
  const double* x0;
  __device__ uint32_t a(int i) const { return adj[i]; }
  __device__ double x(int i) const { return x0[2 * i]; }
  __device__ double y(int i) const { return x0[2 * i + 1]; }
};

struct StagedRow {
  const uint32_t* adj;  // &adj_l[0][lane]
  const double* x0;     // &x0_l[0][lane]
  __device__ uint32_t a(int i) const { return adj[i * kSortBlock]; }
  __device__ double x(int i) const { return x0[(2 * i) * kSortBlock]; }
  __device__ double y(int i) const { return x0[(2 * i + 1) * kSortBlock]; }
};

// squared distance written as (x_i - x_j)^2 + (y_i - y_j)^2, the reference's operation order
template <typename Row>
__device__ inline double sqd(const Row& r, int i, int j) {
  const double dx = r.x(i) - r.x(j);
  const double dy = r.y(i) - r.y(j);
  return dx * dx + dy * dy;
}

// Integer structure of one candidate (the rules links_solve_order documents).
template <typename Row>
__device__ bool structure_ok(int J, int n, const Row& r, uint32_t fixed, int pivot, int tip) {
  if (n < 3 || n > J) return false;
  const uint32_t live = live_mask(n);
  if (fixed & ~live) return false;
  for (int i = 0; i < J; i++) {
    const uint32_t ri = r.a(i);
    if (i >= n) {
      if (ri) return false;
      continue;
    }
    if ((ri & ~live) || ((ri >> i) & 1u)) return false;
    for (uint32_t m = ri; m; m &= m - 1u)
      if (!((r.a(lowbit(m)) >> i) & 1u)) return false;
  }
  if (pivot >= n || tip >= n || pivot == tip) return false;
  if (!((fixed >> pivot) & 1u) || ((fixed >> tip) & 1u) || !((r.a(pivot) >> tip) & 1u)) return false;
  return true;
}

// Finite positions and links longer than 1e-12; scale = longest link; counts the
// links that are not between two fixed joints.
template <typename Row>
__device__ bool geometry_ok(int n, const Row& r, uint32_t fixed, double* scale, int* movable_links) {
  for (int i = 0; i < n; i++)
    if (!isfinite(r.x(i)) || !isfinite(r.y(i))) return false;
  double sc = 0.0;
  int m = 0;
  bool ok = true;
  for (int i = 0; i < n; i++)
    for (uint32_t b = r.a(i) & ~((2u << i) - 1u); b; b &= b - 1u) {
      const int j = lowbit(b);
      const double L = sqrt(sqd(r, i, j));
      if (!(L > 1e-12)) ok = false;
      if (L > sc) sc = L;
      if (!(((fixed >> i) & 1u) && ((fixed >> j) & 1u))) m++;
    }
  *scale = sc;
  *movable_links = m;
  return ok;
}

// Rounds of the graphical solver.  When ord != nullptr the entries are stored as
// (k | a << 8 | b << 16) in ord[s * stride] and the entry index of joint k in
// idx[k * stride].  Returns true when every joint is placed.
template <typename Row>
__device__ bool solve_rounds(int n, const Row& r, uint32_t fixed, int tip, uint32_t* ord, uint8_t* idx,
                             int stride, int* nd_out, int* depth_out) {
  uint32_t known = fixed | (1u << tip);
  int nd = 0, depth = 0;
  for (;;) {
    uint32_t now = 0u;
    for (int k = 0; k < n; k++) {
      if ((known >> k) & 1u) continue;
      const uint32_t kn = r.a(k) & known;
      if (popc(kn) < 2) continue;
      if (ord) {
        const int a = lowbit(kn);
        const int b = lowbit(kn & (kn - 1u));
        ord[nd * stride] = (uint32_t)k | ((uint32_t)a << 8) | ((uint32_t)b << 16);
        idx[k * stride] = (uint8_t)nd;
      }
      nd++;
      now |= 1u << k;
    }
    if (!now) break;
    known |= now;
    depth++;
  }
  *nd_out = nd;
  *depth_out = depth;
  return known == live_mask(n);
}

// The same three analyses with the candidate's rows held in registers (JM >= J
// joints, rows and positions beyond the candidate's joints zero): every loop over
// joints is unrolled, so no row is read at a run-time index, and the decisions are
// those of structure_ok, geometry_ok and solve_rounds.
template <int JM>
__device__ bool reg_structure_ok(int J, int n, const uint32_t (&R)[JM], uint32_t fixed, int pivot, int tip) {
  if (n < 3 || n > J) return false;
  if (pivot >= n || tip >= n || pivot == tip) return false;
  const uint32_t live = live_mask(n);
  bool ok = (fixed & ~live) == 0u;
  uint32_t asym = 0u;  // bit 0: some pair (i, j) linked one way only
  uint32_t rp = 0u;    // row of the pivot
#pragma unroll
  for (int i = 0; i < JM; i++) {
    const uint32_t ri = R[i];
    if (i >= n)
      ok &= ri == 0u;
    else
      ok &= (ri & ~live) == 0u && !((ri >> i) & 1u);
#pragma unroll
    for (int j = i + 1; j < JM; j++) asym |= (ri >> j) ^ (R[j] >> i);
    rp = i == pivot ? ri : rp;
    __builtin_amdgcn_sched_barrier(0);
  }
  ok &= (asym & 1u) == 0u;
  ok &= ((fixed >> pivot) & 1u) && !((fixed >> tip) & 1u) && ((rp >> tip) & 1u);
  return ok;
}

// Link lengths are compared through their squares: the square root is monotone
// and correctly rounded, so the longest link is sqrt of the largest square, and a
// link exceeds 1e-12 exactly when its square exceeds len2_min, the largest double
// whose square root is at most 1e-12.  Every pair of joints is visited (no row is
// read at a run-time index); a pair without a link contributes a square whose high
// word is cleared, a value below 2^-1041 that never exceeds the actuator link's
// (which a structurally valid candidate always has).
template <int JM>
__device__ bool reg_geometry_ok(int n, const uint32_t (&R)[JM], const double (&X)[JM], const double (&Y)[JM],
                                uint32_t fixed, double len2_min, double* scale, int* movable) {
  bool fin = true;
#pragma unroll
  for (int i = 0; i < JM; i++)
    if (i < n) fin &= isfinite(X[i]) && isfinite(Y[i]);
  if (!fin) return false;
  double dmax = 0.0;
  bool short_link = false;
  int m = 0;
#pragma unroll
  for (int i = 0; i < JM; i++) {
    const uint32_t above = R[i] & ~((2u << i) - 1u);  // links to higher joints
    m += popc(((fixed >> i) & 1u) ? (above & ~fixed) : above);
#pragma unroll
    for (int j = i + 1; j < JM; j++) {
      const bool e = (R[i] >> j) & 1u;
      const double dx = X[i] - X[j];
      const double dy = Y[i] - Y[j];
      const double d2 = dx * dx + dy * dy;
      dmax = fmax(dmax, __hiloint2double(e ? __double2hiint(d2) : 0, __double2loint(d2)));
      short_link = short_link | (e & !(d2 > len2_min));
    }
    __builtin_amdgcn_sched_barrier(0);  // one row at a time: bounded register pressure
  }
  *scale = sqrt(dmax);
  *movable = m;
  return !short_link;
}

// Rounds of the graphical solver; with ord != nullptr the entries and the entry
// index of every placed joint are stored as solve_rounds stores them.
template <int JM>
__device__ bool reg_solve_rounds(int n, const uint32_t (&R)[JM], uint32_t fixed, int tip, uint32_t* ord,
                                 uint8_t* idx, int stride, int* nd_out) {
  uint32_t known = fixed | (1u << tip);
  int nd = 0;
  for (;;) {
    uint32_t now = 0u;
#pragma unroll
    for (int k = 0; k < JM; k++) {
      const uint32_t kn = R[k] & known;
      const bool place = k < n && !((known >> k) & 1u) && popc(kn) >= 2;
      if (ord && place) {
        const int a = lowbit(kn);
        const int b = lowbit(kn & (kn - 1u));
        ord[nd * stride] = (uint32_t)k | ((uint32_t)a << 8) | ((uint32_t)b << 16);
        idx[k * stride] = (uint8_t)nd;
      }
      nd += place ? 1 : 0;
      now |= place ? (1u << k) : 0u;
    }
    if (!now) break;
    known |= now;
  }
  *nd_out = nd;
  return known == live_mask(n);
}

// joints-per-candidate class of the register-resident kernels
__host__ __device__ inline int jm_class(int J) {
  return J <= 8 ? 8 : J <= 12 ? 12 : J <= 16 ? 16 : J <= 20 ? 20 : J <= 24 ? 24 : 32;
}

// Copies the workgroup's adjacency rows and initial positions into LDS, lanes
// interleaved, with coalesced loads (the rows of consecutive candidates are
// contiguous in memory).  The loads of kStageUnroll elements per lane are issued
// together before any of them is stored.  Every thread of the workgroup must call it.
constexpr int kStageUnroll = 8;

__device__ StagedRow stage_rows(const PrepArgs& A, unsigned char* smem) {
  const int J = A.J;
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * kSortBlock;
  const int nc = min(kSortBlock, A.B - c0);
  uint32_t* adj_l = reinterpret_cast<uint32_t*>(smem);                          // [J][64]
  double* x0_l = reinterpret_cast<double*>(smem + (size_t)J * kSortBlock * 4);  // [2J][64]
  const uint32_t* ag = A.adj + (size_t)c0 * J;
  const double2* xg = reinterpret_cast<const double2*>(A.x0 + (size_t)c0 * J * 2);
  const int total = nc * J;  // >= 3: the workgroup holds at least one candidate
  for (int e0 = tid; e0 < total; e0 += kStageUnroll * kSortBlock) {
    uint32_t av[kStageUnroll];
    double2 xv[kStageUnroll];
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const int e = min(e0 + u * kSortBlock, total - 1);  // in bounds; the extra loads are not stored
      av[u] = ag[e];
      xv[u] = xg[e];
    }
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const int e = e0 + u * kSortBlock;
      if (e < total) {
        const int cand = e / J, i = e - cand * J;
        adj_l[i * kSortBlock + cand] = av[u];
        x0_l[(2 * i) * kSortBlock + cand] = xv[u].x;
        x0_l[(2 * i + 1) * kSortBlock + cand] = xv[u].y;
      }
    }
  }
  __syncthreads();
  StagedRow r;
  r.adj = adj_l + tid;
  r.x0 = x0_l + tid;
  return r;
}

// The same copy in parts, for the register-resident count pass: the adjacency
// rows ([J][64] u32), then kPosPart joints of the positions at a time ([2 kPosPart][64]
// f64), each part through the same LDS buffer, so that a workgroup holds 8 KB of
// LDS rather than 20 J bytes per lane and more workgroups share a CU.
constexpr int kPosPart = 8;

__host__ __device__ inline size_t parts_bytes(int J) {
  const size_t a = (size_t)J * kSortBlock * 4, x = (size_t)kPosPart * kSortBlock * 16;
  return a > x ? a : x;
}

__device__ void stage_adj(const PrepArgs& A, uint32_t* adj_l) {
  const int J = A.J;
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * kSortBlock;
  const int nc = min(kSortBlock, A.B - c0);
  const uint32_t* ag = A.adj + (size_t)c0 * J;
  const int total = nc * J;
  for (int e0 = tid; e0 < total; e0 += kStageUnroll * kSortBlock) {
    uint32_t av[kStageUnroll];
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) av[u] = ag[min(e0 + u * kSortBlock, total - 1)];
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const int e = e0 + u * kSortBlock;
      if (e < total) {
        const int cand = e / J, i = e - cand * J;
        adj_l[i * kSortBlock + cand] = av[u];
      }
    }
  }
}

// joints j0 .. j0 + nj - 1 (nj <= kPosPart) of every candidate of the workgroup
__device__ void stage_pos_part(const PrepArgs& A, double* x_l, int j0, int nj) {
  const int J = A.J;
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * kSortBlock;
  const int nc = min(kSortBlock, A.B - c0);
  const double2* xg = reinterpret_cast<const double2*>(A.x0 + (size_t)c0 * J * 2);
  const int total = nc * nj;
  constexpr int U = kStageUnroll / 2;  // the positions of earlier parts are held in registers meanwhile
  for (int e0 = tid; e0 < total; e0 += U * kSortBlock) {
    double2 xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = min(e0 + u * kSortBlock, total - 1);
      const int cand = e / nj, i = e - cand * nj;
      xv[u] = xg[(size_t)cand * J + j0 + i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kSortBlock;
      if (e < total) {
        const int cand = e / nj, i = e - cand * nj;
        x_l[(2 * i) * kSortBlock + cand] = xv[u].x;
        x_l[(2 * i + 1) * kSortBlock + cand] = xv[u].y;
      }
    }
  }
}

__global__ void __launch_bounds__(kPrepBlock) solve_order_kernel(PrepArgs A) {
  __shared__ uint32_t ord_l[kMaxJ * kPrepBlock];
  __shared__ uint8_t idx_l[kMaxJ * kPrepBlock];
  const int tid = threadIdx.x;
  const int c = blockIdx.x * blockDim.x + tid;
  if (c >= A.B) return;
  const int J = A.J;
  const int n = A.n[c];
  GlobalRow row;
  row.adj = A.adj + (size_t)c * J;
  row.x0 = nullptr;
  const uint32_t fixed = A.fixed[c];
  const int pivot = A.motor[2 * c], tip = A.motor[2 * c + 1];
  const bool ok = structure_ok(J, n, row, fixed, pivot, tip);
  int nd = 0, depth = 0;
  bool complete = false;
  if (ok) complete = solve_rounds(n, row, fixed, tip, ord_l + tid, idx_l + tid, kPrepBlock, &nd, &depth);
  if (A.order) {
    int8_t* o = A.order + (size_t)c * J * 3;
    for (int s = 0; s < J; s++) {
      const bool has = ok && s < nd;
      const uint32_t e = has ? ord_l[s * kPrepBlock + tid] : 0u;
      o[3 * s + 0] = has ? (int8_t)(e & 0xFF) : (int8_t)-1;
      o[3 * s + 1] = has ? (int8_t)((e >> 8) & 0xFF) : (int8_t)-1;
      o[3 * s + 2] = has ? (int8_t)((e >> 16) & 0xFF) : (int8_t)-1;
    }
  }
  if (A.n_dyads) A.n_dyads[c] = ok ? (uint8_t)nd : 0;
  if (A.depth) A.depth[c] = ok ? (uint8_t)depth : 0;
  A.status[c] = !ok ? 5 : (complete ? 0 : 4);
}

// ---- simulation set-up, pass 1: status of malformed / unsolvable candidates,
// solve-order length D of the others and a per-workgroup histogram of D.  The
// rows are staged through LDS with coalesced loads and then held in registers.
template <int JM>
__global__ void __launch_bounds__(kSortBlock) count_kernel(PrepArgs A) {
  extern __shared__ unsigned char smem[];
  const int tid = threadIdx.x;
  const int c = blockIdx.x * kSortBlock + tid;
  const bool in = c < A.B;
  // per-candidate scalars, loaded before the rows so that the latencies overlap
  const int n = in ? A.n[c] : 0;
  const uint32_t fixed = in ? A.fixed[c] : 0u;
  const int pivot = in ? A.motor[2 * c] : 0, tip = in ? A.motor[2 * c + 1] : 0;
  const bool prev_rejected = in && A.pre_ratio > 0 && A.status[c] != 0;
  const int J = A.J;
  uint32_t R[JM];
  double X[JM], Y[JM];
  StagedRow row;  // above 24 joints: rows and positions read from LDS
  row.adj = nullptr;
  row.x0 = nullptr;
  if (JM < 32) {
    // rows, then the positions a part at a time, into registers
    uint32_t* adj_l = reinterpret_cast<uint32_t*>(smem);
    double* x_l = reinterpret_cast<double*>(smem);
    stage_adj(A, adj_l);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < JM; i++) R[i] = i < J ? adj_l[i * kSortBlock + tid] : 0u;
#pragma unroll
    for (int j0 = 0; j0 < JM; j0 += kPosPart) {
      if (j0 < J) {
        const int nj = min(kPosPart, J - j0);
        __syncthreads();  // the buffer's previous contents have been read
        stage_pos_part(A, x_l, j0, nj);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPosPart; k++) {
          const int i = j0 + k;
          if (i < JM) {
            const bool have = i < J && i < n;
            X[i] = have ? x_l[(2 * k) * kSortBlock + tid] : 0.0;
            Y[i] = have ? x_l[(2 * k + 1) * kSortBlock + tid] : 0.0;
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < kPosPart; k++)
          if (j0 + k < JM) X[j0 + k] = Y[j0 + k] = 0.0;
      }
    }
  } else {
    row = stage_rows(A, smem);
#pragma unroll
    for (int i = 0; i < JM; i++) R[i] = i < J ? row.a(i) : 0u;
  }
  int dl = 0xFF;
  if (prev_rejected) {
    // rejected by the low-fidelity pass: keep its decision, on the fine grid
    const int fs = A.fail_step[c];
    if (fs >= 0) A.fail_step[c] = (int16_t)(fs * A.pre_ratio);
    if (A.esc_step) A.esc_step[c] = -1;
    A.dlen[c] = 0xFF;
  }
  if (in && !prev_rejected) {
    // the decisions do not depend on one another's order: integer ones first,
    // then the positions for the geometry
    bool ok = JM < 32 ? reg_structure_ok<JM>(J, n, R, fixed, pivot, tip) : structure_ok(J, n, row, fixed, pivot, tip);
    int nd = 0;
    bool complete = false;
    if (ok) complete = reg_solve_rounds<JM>(n, R, fixed, tip, nullptr, nullptr, 0, &nd);
    double scale = 0.0;
    int movable = 0;
    if (ok && JM == 32) {
      ok = geometry_ok(n, row, fixed, &scale, &movable);
    } else if (ok) {
      ok = reg_geometry_ok<JM>(n, R, X, Y, fixed, A.len2_min, &scale, &movable);
    }
    uint8_t st = !ok ? 5 : (complete ? kPending : 4);
    A.status[c] = st;
    dl = st == kPending ? nd : 0xFF;
    A.dlen[c] = (uint8_t)dl;
    if (st == kPending) {
      // handed to the fill pass, which reads them at the sorted position
      A.scale_ws[c] = scale;
      A.movable_ws[c] = (int16_t)movable;
    } else {
      A.fail_step[c] = -1;
      if (A.esc_step) A.esc_step[c] = -1;
    }
  }
  // histogram of D over the workgroup (one wave), stored by bucket: [32][blocks]
  for (int d = 0; d < kMaxJ; d++) {
    const int k = __popcll(__ballot(dl == d));
    if (tid == d) A.block_hist[(size_t)d * gridDim.x + blockIdx.x] = k;
  }
}

// pass 2: exclusive scan of every bucket's per-workgroup counts (one workgroup per
// D, reading the bucket's row of [32][blocks] a tile of 1024 at a time): a scan
// within each wave, then over the 16 wave totals
__global__ void __launch_bounds__(1024) offsets_kernel(int32_t nblocks, const int32_t* block_hist,
                                                        int32_t* block_off, int32_t* counters) {
  __shared__ int32_t wsum[16];
  const int d = blockIdx.x;
  const int32_t* h = block_hist + (size_t)d * nblocks;
  int32_t* o = block_off + (size_t)d * nblocks;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int carry = 0;
  for (int base = 0; base < nblocks; base += 1024) {
    const int i = base + threadIdx.x;
    const int v = i < nblocks ? h[i] : 0;
    int x = v;  // inclusive scan within the wave
#pragma unroll
    for (int k = 1; k < kWave; k <<= 1) {
      const int y = __shfl_up(x, k);
      if (lane >= k) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) {
      const int t = wsum[k];
      pre += k < w ? t : 0;
      tot += t;
    }
    if (i < nblocks) o[i] = carry + pre + x - v;
    carry += tot;
    __syncthreads();  // wsum is rewritten by the next tile
  }
  if (threadIdx.x == 0) counters[kCntHist + d] = carry;
}

// pass 2b: bucket starts, largest D first, and the work counters
__global__ void starts_kernel(int32_t* counters) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t off = 0;
  for (int d = kMaxJ - 1; d >= 0; d--) {
    counters[kCntOff + d] = off;
    counters[kCntCur + d] = off;
    off += counters[kCntHist + d];
  }
  counters[kCntItems] = off;
  counters[kCntNext] = 0;
}

// pass 3: position of every pending candidate in the sorted work list (largest D
// first, candidate index within a bucket).
__global__ void __launch_bounds__(kSortBlock) rank_kernel(PrepArgs A) {
  const int tid = threadIdx.x;
  const int c = blockIdx.x * kSortBlock + tid;
  const int myd = c < A.B ? A.dlen[c] : 0xFF;
  // rank among the lanes of this workgroup (one wave) with the same D
  const uint64_t below = tid == 0 ? 0ull : (~0ull >> (64 - tid));
  int rank = 0;
  for (int d = 0; d < kMaxJ; d++) {
    const uint64_t m = __ballot(myd == d);
    if (myd == d) rank = __popcll(m & below);
  }
  if (myd == 0xFF) return;
  const int p = A.counters[kCntOff + myd] + A.block_off[(size_t)myd * gridDim.x + blockIdx.x] + rank;
  A.perm[p] = c;
}

// pass 4: the records of the candidate at every sorted position p.  Each lane
// gathers its candidate's rows into its own LDS column, so the record writes of a
// wave go to consecutive positions.
template <int JM>
__global__ void __launch_bounds__(kSortBlock) fill_kernel(PrepArgs A) {
  extern __shared__ unsigned char smem[];
  __shared__ uint32_t ord_l[JM * kSortBlock];
  __shared__ uint8_t idx_l[JM * kSortBlock];
  const int tid = threadIdx.x;
  const int p = blockIdx.x * kSortBlock + tid;
  if (p >= A.counters[kCntItems]) return;
  const int c = A.perm[p];
  const int J = A.J;
  // the candidate's scalars and rows, every load issued before the first store
  const int n = A.n[c];
  const uint32_t fixed = A.fixed[c];
  const int pivot = A.motor[2 * c], tip = A.motor[2 * c + 1];
  // scale and movable-link count as the count pass found them
  const double scale = A.scale_ws[c];
  const int movable = A.movable_ws[c];
  const uint32_t* ag = A.adj + (size_t)c * J;
  uint32_t R[JM];
#pragma unroll
  for (int i = 0; i < JM; i++) R[i] = ag[min(i, J - 1)];  // in the row; rows >= J cleared below
#pragma unroll
  for (int i = 0; i < JM; i++) R[i] = i < J ? R[i] : 0u;
  StagedRow row;
  {
    double* x0_l = reinterpret_cast<double*>(smem);  // [2 JM][64]
    const double2* xg = reinterpret_cast<const double2*>(A.x0 + (size_t)c * J * 2);
    double2 xv[JM];
#pragma unroll
    for (int i = 0; i < JM; i++) xv[i] = xg[min(i, n - 1)];
#pragma unroll
    for (int i = 0; i < JM; i++)
      if (i < n) {
        x0_l[(2 * i) * kSortBlock + tid] = xv[i].x;
        x0_l[(2 * i + 1) * kSortBlock + tid] = xv[i].y;
      }
    row.adj = nullptr;
    row.x0 = x0_l + tid;
  }

  const int Bs = A.Bs;
  int nd = 0;
  reg_solve_rounds<JM>(n, R, fixed, tip, ord_l + tid, idx_l + tid, kSortBlock, &nd);
  const int D = nd;
  // links outside the solve order: all but the actuator arm and two per placed joint
  const int redundant = movable - 1 - 2 * nd;
  auto slot_of = [&](int j) -> int {
    if (j == tip) return D;
    if ((fixed >> j) & 1u) return D + 1 + popc(fixed & ((1u << j) - 1u));
    return idx_l[j * kSortBlock + tid];
  };
  CandMeta m;
  m.D = (uint8_t)D;
  m.n = (uint8_t)n;
  int out = A.out_joint;
  uint32_t flags = redundant > 0 ? kFlagRedundant : 0u;
  if (out < 0) out = D > 0 ? (int)(ord_l[(D - 1) * kSortBlock + tid] & 0xFF) : tip;
  if (out >= n) {
    flags |= kFlagNoPath;
    m.out_slot = 0;
  } else {
    m.out_slot = (uint8_t)slot_of(out);
  }
  m.flags = (uint8_t)flags;
  A.meta[p] = m;
  A.perm[p] = c;

  // starting side of every placed joint (bit s: left of a->b, ties left), the
  // oracle's cross product evaluated in the same order
  uint32_t side = 0u;
  for (int s = 0; s < D; s++) {
    const uint32_t e = ord_l[s * kSortBlock + tid];
    const int k = e & 0xFF, a = (e >> 8) & 0xFF, b = (e >> 16) & 0xFF;
    const double cr = (row.x(b) - row.x(a)) * (row.y(k) - row.y(a)) - (row.y(b) - row.y(a)) * (row.x(k) - row.x(a));
    side |= cr >= 0.0 ? (1u << s) : 0u;
  }
  const double px = row.x(pivot), py = row.y(pivot);
  const double vx = row.x(tip) - px, vy = row.y(tip) - py;
  const double scale2 = scale * scale;
  CandF64 cd;
  cd.px = px;
  cd.py = py;
  cd.vx = vx;
  cd.vy = vy;
  cd.scale = scale;
  cd.deg_thr = 1e-12 * scale2;
  cd.drift_thr = A.tau_drift * scale;
  cd.side = side;
  A.cd[p] = cd;

  // FP32 thresholds and error units: a computed position carries at most a few
  // units of FP32 rounding of its magnitude before amplification
  const double u = (double)kRoundUnit;
  CandF32 cf;
  cf.px = (float)px;
  cf.py = (float)py;
  cf.vx = (float)vx;
  cf.vy = (float)vy;
  cf.U = (float)(u * (fabs(px) + fabs(py) + fabs(vx) + fabs(vy)));
  cf.KB = (float)(4.0 * A.eps_disc * scale2 * scale2);
  cf.CD = (float)(A.eps_disc * scale2);
  cf.EB = (float)(A.eps_branch * scale);
  cf.U2 = (float)(u * 2.0 * scale);
  cf.TS = (float)(2.0 * scale);
  cf.u = (float)u;
  cf.DG = (float)(1e-12 * scale2);
  cf.side = side;
  cf.pad[0] = cf.pad[1] = cf.pad[2] = 0.f;
  A.cf[p] = cf;

  for (int s = 0; s < D; s++) {
    const uint32_t e = ord_l[s * kSortBlock + tid];
    const int k = e & 0xFF, a = (e >> 8) & 0xFF, b = (e >> 16) & 0xFF;
    const double ra2 = sqd(row, k, a);
    const double rb2 = sqd(row, k, b);
    const double ra = sqrt(ra2), rb = sqrt(rb2);
    const double sum = ra + rb, dif = ra - rb;
    DyadF64 q;
    q.ra2 = ra2;
    q.rb2 = rb2;
    q.S = sum * sum;
    q.Dm = dif * dif;
    A.dd[(size_t)s * Bs + p] = q;
    DyadF32 f;
    f.S = (float)(sum * sum);
    f.Dm = (float)(dif * dif);
    f.Kc = (float)(0.5 * (ra2 - rb2));
    f.slots = (uint32_t)slot_of(a) | ((uint32_t)slot_of(b) << 8);
    A.df[(size_t)s * Bs + p] = f;
  }
  for (int j = 0; j < n; j++) {
    const int sl = slot_of(j);
    A.x0s[(size_t)sl * Bs + p] = make_float2((float)row.x(j), (float)row.y(j));
    A.slot_joint[(size_t)sl * Bs + p] = (uint8_t)j;
  }
}

__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// ---- compaction of valid candidates (ascending candidate index)
constexpr int kScanBlock = 256;

__global__ void __launch_bounds__(kScanBlock) count_valid_kernel(int32_t B, const uint8_t* status,
                                                                  int32_t* block_counts) {
  __shared__ int32_t s[kScanBlock];
  int c = blockIdx.x * kScanBlock + threadIdx.x;
  s[threadIdx.x] = (c < B && status[c] == 0) ? 1 : 0;
  __syncthreads();
  for (int w = kScanBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_counts[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(1024) scan_blocks_kernel(int32_t nblocks, int32_t* block_counts,
                                                           int32_t* total) {
  // single block; sequential chunks of 1024 with a running carry
  __shared__ int32_t s[1024];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nblocks; base += 1024) {
    int i = base + threadIdx.x;
    int v = i < nblocks ? block_counts[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = 1; w < 1024; w <<= 1) {
      int add = threadIdx.x >= w ? s[threadIdx.x - w] : 0;
      __syncthreads();
      s[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nblocks) block_counts[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(kScanBlock) write_index_kernel(int32_t B, const uint8_t* status,
                                                                  const int32_t* block_offsets,
                                                                  int32_t* index, int32_t cap, int32_t* row_of) {
  __shared__ int32_t s[kScanBlock];
  int c = blockIdx.x * kScanBlock + threadIdx.x;
  int v = (c < B && status[c] == 0) ? 1 : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int w = 1; w < kScanBlock; w <<= 1) {
    int add = threadIdx.x >= w ? s[threadIdx.x - w] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  int pos = block_offsets[blockIdx.x] + s[threadIdx.x] - v;
  if (v && pos < cap) index[pos] = c;
  if (v && row_of) row_of[c] = pos < cap ? pos : -1;
}

// selection of the path list over sorted positions p < items
__device__ inline int path_flag(int p, int items, const int32_t* perm, const uint8_t* status,
                                const int32_t* row_of, int all_simulated) {
  if (p >= items) return 0;
  const int c = perm[p];
  if (all_simulated) return status[c] <= 3 ? 1 : 0;
  return (status[c] == 0 && row_of[c] >= 0) ? 1 : 0;
}

__global__ void __launch_bounds__(kScanBlock) count_sel_kernel(const int32_t* counters, const int32_t* perm,
                                                                const uint8_t* status, const int32_t* row_of,
                                                                int all_simulated, int32_t* block_counts) {
  __shared__ int32_t s[kScanBlock];
  const int p = blockIdx.x * kScanBlock + threadIdx.x;
  s[threadIdx.x] = path_flag(p, counters[kCntItems], perm, status, row_of, all_simulated);
  __syncthreads();
  for (int w = kScanBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_counts[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(kScanBlock) write_sel_kernel(const int32_t* counters, const int32_t* perm,
                                                                const uint8_t* status, const int32_t* row_of,
                                                                int all_simulated, const int32_t* block_offsets,
                                                                int32_t* list) {
  __shared__ int32_t s[kScanBlock];
  const int p = blockIdx.x * kScanBlock + threadIdx.x;
  const int v = path_flag(p, counters[kCntItems], perm, status, row_of, all_simulated);
  s[threadIdx.x] = v;
  __syncthreads();
  for (int w = 1; w < kScanBlock; w <<= 1) {
    const int add = threadIdx.x >= w ? s[threadIdx.x - w] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  if (v) list[block_offsets[blockIdx.x] + s[threadIdx.x] - v] = p;
}


// Curation (Methodology, "Dataset Curation & Processing"), one wave per path: the
// variance of the distances of the DIAMETER-normalised path from the centre of the
// unit box (circles have none), whether the path's joint is linked to a ground
// joint (it then turns on an arc about it), and the joints the path's joint depends
// on through the solve order (the reduced mechanism).
constexpr int kCurateBlock = 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__global__ void __launch_bounds__(kCurateBlock) curate_kernel(CurateArgs a) {
  __shared__ uint32_t ord[kMaxJ];
  __shared__ uint8_t idx[kMaxJ];
  const int i = blockIdx.x;
  const int rows = a.count ? min(*a.count, a.cap) : a.cap;
  if (i >= rows) return;  // uniform over the workgroup
  const int lane = threadIdx.x;
  const int T = a.T;
  const float2* q = reinterpret_cast<const float2*>(a.norm) + (size_t)i * T;
  double s = 0.0;
  for (int t = lane; t < T; t += kCurateBlock) {
    const float2 p = q[t];
    const double dx = (double)p.x - 0.5, dy = (double)p.y - 0.5;
    s += sqrt(dx * dx + dy * dy);
  }
  const double mean = wave_sum(s) / (double)T;
  double v = 0.0;
  for (int t = lane; t < T; t += kCurateBlock) {
    const float2 p = q[t];
    const double dx = (double)p.x - 0.5, dy = (double)p.y - 0.5;
    const double e = sqrt(dx * dx + dy * dy) - mean;
    v += e * e;
  }
  const double var = wave_sum(v) / (double)T;
  if (lane != 0) return;
  const int c = a.path_index ? a.path_index[i] : i;
  a.radial_var[i] = (float)var;
  GlobalRow row;
  row.adj = a.adj + (size_t)c * a.J;
  row.x0 = nullptr;
  const uint32_t fixed = a.fixed[c];
  const int pivot = a.motor[2 * c], tip = a.motor[2 * c + 1];
  int nd = 0, depth = 0;
  uint32_t f = 0u, keep = 0u;
  if (structure_ok(a.J, a.n[c], row, fixed, pivot, tip) &&
      solve_rounds(a.n[c], row, fixed, tip, ord, idx, 1, &nd, &depth)) {
    const int out = a.out_joint >= 0 ? a.out_joint : (nd > 0 ? (int)(ord[nd - 1] & 0xFF) : tip);
    if (row.a(out) & fixed) f |= 1u;         // arc
    if (var < a.circle_var) f |= 2u;         // circle
    keep = 1u << out;
    for (int k = nd - 1; k >= 0; k--) {
      const uint32_t e = ord[k];
      if ((keep >> (e & 0xFF)) & 1u) keep |= (1u << ((e >> 8) & 0xFF)) | (1u << ((e >> 16) & 0xFF));
    }
    if ((keep >> tip) & 1u) keep |= 1u << pivot;
  }
  a.flags[i] = (uint8_t)f;
  a.keep[i] = keep;
}

}  // namespace

hipError_t launch_curate(const CurateArgs& a, hipStream_t st) {
  if (a.cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(curate_kernel, dim3(a.cap), dim3(kCurateBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_solve_order(const PrepArgs& a, hipStream_t st) {
  if (a.B <= 0) return hipSuccess;
  const int grid = (a.B + kPrepBlock - 1) / kPrepBlock;
  hipLaunchKernelGGL(solve_order_kernel, dim3(grid), dim3(kPrepBlock), 0, st, a);
  return hipGetLastError();
}

int prep_blocks(int32_t B) { return (B + kSortBlock - 1) / kSortBlock; }

// LDS of the staged rows: adjacency [J][64] u32 and positions [2J][64] f64
size_t staged_bytes(int J) { return (size_t)J * kSortBlock * (4 + 16); }
// LDS of the fill pass's positions [2J][64] f64
size_t fill_bytes(int J) { return (size_t)J * kSortBlock * 16; }

template <int JM>
void count_one(const PrepArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(count_kernel<JM>, dim3(prep_blocks(a.B)), dim3(kSortBlock),
                     JM < 32 ? parts_bytes(a.J) : staged_bytes(a.J), st, a);
}

hipError_t launch_prep_count(const PrepArgs& a, hipStream_t st) {
  if (a.B <= 0) return hipSuccess;
  switch (jm_class(a.J)) {
    case 8: count_one<8>(a, st); break;
    case 12: count_one<12>(a, st); break;
    case 16: count_one<16>(a, st); break;
    case 20: count_one<20>(a, st); break;
    case 24: count_one<24>(a, st); break;
    default: count_one<32>(a, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_prep_offsets(const PrepArgs& a, hipStream_t st) {
  const int nb = prep_blocks(a.B);
  if (nb > 0) hipLaunchKernelGGL(offsets_kernel, dim3(kMaxJ), dim3(1024), 0, st, nb, a.block_hist, a.block_off,
                                 a.counters);
  hipLaunchKernelGGL(starts_kernel, dim3(1), dim3(64), 0, st, a.counters);
  return hipGetLastError();
}

hipError_t launch_prep_fill(const PrepArgs& a, hipStream_t st) {
  if (a.B <= 0) return hipSuccess;
  hipLaunchKernelGGL(rank_kernel, dim3(prep_blocks(a.B)), dim3(kSortBlock), 0, st, a);
  const dim3 g(prep_blocks(a.B)), b(kSortBlock);
  switch (jm_class(a.J)) {
    case 8: hipLaunchKernelGGL(fill_kernel<8>, g, b, fill_bytes(a.J), st, a); break;
    case 12: hipLaunchKernelGGL(fill_kernel<12>, g, b, fill_bytes(a.J), st, a); break;
    case 16: hipLaunchKernelGGL(fill_kernel<16>, g, b, fill_bytes(a.J), st, a); break;
    case 20: hipLaunchKernelGGL(fill_kernel<20>, g, b, fill_bytes(a.J), st, a); break;
    case 24: hipLaunchKernelGGL(fill_kernel<24>, g, b, fill_bytes(a.J), st, a); break;
    default: hipLaunchKernelGGL(fill_kernel<32>, g, b, fill_bytes(a.J), st, a); break;
  }
  return hipGetLastError();
}

__global__ void resume_setup_kernel(const int32_t* counters, int32_t* counters2) {
  const int i = threadIdx.x;
  for (int k = i; k < kCntSize; k += blockDim.x) counters2[k] = 0;
  __syncthreads();
  if (i == 0) {
    const int r = counters[kCntRes];
    counters2[kCntHist + 0] = r;
    counters2[kCntItems] = r;
  }
}

hipError_t launch_resume_setup(const int32_t* counters, int32_t* counters2, hipStream_t st) {
  hipLaunchKernelGGL(resume_setup_kernel, dim3(1), dim3(128), 0, st, counters, counters2);
  return hipGetLastError();
}

__global__ void widen_kernel(const float* in, double* out, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) out[i] = (double)in[i];
}

hipError_t launch_widen(const float* in, double* out, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const size_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(widen_kernel, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

hipError_t launch_fill_u32(void* p, size_t n_u32, uint32_t v, hipStream_t st) {
  if (n_u32 == 0) return hipSuccess;
  size_t blocks = (n_u32 + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t*)p, n_u32, v);
  return hipGetLastError();
}

size_t compact_scratch_ints(int32_t B) { return (size_t)((B + kScanBlock - 1) / kScanBlock) + 1; }

// ---- the hand-over queue ordered by hand-over step, earliest first: a candidate
// handed over early may have the most FP64 steps ahead of it, so the FP64 pass
// starts those first and its last waves are not left with long runs.  Key = the
// step / 8 (at most kEscBins keys); entries with equal keys keep no particular
// order (each is a candidate of its own).
constexpr int kEscBlock = 1024;

__global__ void __launch_bounds__(kEscBlock) esc_hist_kernel(const int32_t* counters, const EscEntry* q,
                                                             int32_t* hist) {
  __shared__ int32_t h[kEscBins];
  for (int i = threadIdx.x; i < kEscBins; i += kEscBlock) h[i] = 0;
  __syncthreads();
  const int n = counters[kCntEsc];
  const int i = blockIdx.x * kEscBlock + threadIdx.x;
  if (i < n) atomicAdd(&h[min((int)q[i].t >> 3, kEscBins - 1)], 1);
  __syncthreads();
  for (int k = threadIdx.x; k < kEscBins; k += kEscBlock)
    if (h[k]) atomicAdd(&hist[k], h[k]);
}

__global__ void __launch_bounds__(kEscBlock) esc_scan_kernel(int32_t* hist, int32_t* cursor) {
  // exclusive prefix over kEscBins keys, one block
  __shared__ int32_t part[kEscBlock];
  constexpr int per = kEscBins / kEscBlock;
  const int b = threadIdx.x * per;
  int sum = 0;
  for (int k = 0; k < per; ++k) sum += hist[b + k];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int w = 1; w < kEscBlock; w <<= 1) {
    const int add = threadIdx.x >= w ? part[threadIdx.x - w] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  int run = part[threadIdx.x] - sum;
  for (int k = 0; k < per; ++k) {
    const int c = hist[b + k];
    cursor[b + k] = run;
    run += c;
  }
}

__global__ void __launch_bounds__(kEscBlock) esc_scatter_kernel(const int32_t* counters, const EscEntry* q,
                                                                int32_t* cursor, EscEntry* out) {
  __shared__ int32_t h[kEscBins];
  for (int i = threadIdx.x; i < kEscBins; i += kEscBlock) h[i] = 0;
  __syncthreads();
  const int n = counters[kCntEsc];
  const int i = blockIdx.x * kEscBlock + threadIdx.x;
  int key = 0, rank = 0;
  EscEntry e;
  if (i < n) {
    e = q[i];
    key = min((int)e.t >> 3, kEscBins - 1);
    rank = atomicAdd(&h[key], 1);
  }
  __syncthreads();
  // one range per key of this block
  for (int k = threadIdx.x; k < kEscBins; k += kEscBlock)
    if (h[k]) h[k] = atomicAdd(&cursor[k], h[k]);
  __syncthreads();
  if (i < n) out[h[key] + rank] = e;
}

hipError_t launch_sort_esc(int32_t B, const int32_t* counters, const EscEntry* q, int32_t* work, EscEntry* out,
                           hipStream_t st) {
  if (B <= 0) return hipSuccess;
  int32_t* hist = work;
  int32_t* cursor = work + kEscBins;
  hipError_t e = launch_fill_u32(hist, kEscBins, 0u, st);
  if (e != hipSuccess) return e;
  const int nb = (B + kEscBlock - 1) / kEscBlock;
  hipLaunchKernelGGL(esc_hist_kernel, dim3(nb), dim3(kEscBlock), 0, st, counters, q, hist);
  hipLaunchKernelGGL(esc_scan_kernel, dim3(1), dim3(kEscBlock), 0, st, hist, cursor);
  hipLaunchKernelGGL(esc_scatter_kernel, dim3(nb), dim3(kEscBlock), 0, st, counters, q, cursor, out);
  return hipGetLastError();
}

hipError_t launch_compact(int32_t B, const uint8_t* status, int32_t* scratch, int32_t* index, int32_t cap,
                          int32_t* total, int32_t* row_of, hipStream_t st) {
  int nb = (B + kScanBlock - 1) / kScanBlock;
  if (nb == 0) {
    return launch_fill_u32(total, 1, 0u, st);
  }
  hipLaunchKernelGGL(count_valid_kernel, dim3(nb), dim3(kScanBlock), 0, st, B, status, scratch);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, st, nb, scratch, total);
  hipLaunchKernelGGL(write_index_kernel, dim3(nb), dim3(kScanBlock), 0, st, B, status, scratch, index, cap, row_of);
  return hipGetLastError();
}

hipError_t launch_select_paths(int32_t B, const int32_t* perm, const uint8_t* status, const int32_t* row_of,
                               int all_simulated, int32_t* scratch, int32_t* list, int32_t* counters,
                               hipStream_t st) {
  const int nb = (B + kScanBlock - 1) / kScanBlock;
  if (nb == 0) return launch_fill_u32(counters + kCntPath, 1, 0u, st);
  hipLaunchKernelGGL(count_sel_kernel, dim3(nb), dim3(kScanBlock), 0, st, counters, perm, status, row_of,
                     all_simulated, scratch);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, st, nb, scratch, counters + kCntPath);
  hipLaunchKernelGGL(write_sel_kernel, dim3(nb), dim3(kScanBlock), 0, st, counters, perm, status, row_of,
                     all_simulated, scratch, list);
  return hipGetLastError();
}


}  // namespace links
