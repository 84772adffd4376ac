// sim64.hip -- FP64 simulation passes.
//
// Work sources:
//   kFromPerm  every pending candidate from t = 0 (plain FP64 precision);
//   kFromEsc   the candidates the FP32 pass handed over, from their hand-over step;
//   kFromPath  the candidates whose coupler path is output, from t = 0, writing
//              the path rows (the decision is already taken).
//
// Two arithmetic variants of one step.  EXACT is the sequence of correctly rounded
// double operations below, with no fused multiply-adds (the library is built with
// -ffp-contract=off):
//   tip   = pivot + (cos t * v_x - sin t * v_y, sin t * v_x + cos t * v_y)
//   d^2   = dx*dx + dy*dy                                         (parents a, b)
//   K     = (S - d^2)(d^2 - Dm),  S = (ra+rb)^2, Dm = (ra-rb)^2   (16 area^2, Heron)
//   h     = sqrt(K) / (2 d),  f = (d^2 + ra^2 - rb^2) / (2 d)      (height and its foot)
//   base  = p_a + (f/d)(dx, dy),  off = (h/d)(-dy, dx)
//   p     = base + off or base - off, the one nearer the previous position (tie: +)
// The fast variant evaluates the same intersection with reciprocal square roots
// refined by one Newton step and fused multiply-adds (relative error ~5e-15):
//   1/d = rsq(d^2), alpha = 1/2 + Kc/d^2, beta = sqrt(K)/(2 d^2), Kc = (ra^2-rb^2)/2,
//   base = p_a + alpha (dx, dy), off = beta (-dy, dx), side by the sign of
//   (prev - base) . off.
// A step fails with DEGENERATE when d^2 <= 1e-12 scale^2, LOCKED when K < 0 and
// DRIFT when a link outside the solve order changes length by more than
// tau scale (Methodology, "Finding Valid Initial Positions"; the formulas are the
// textbook circle-circle intersection, which the paper does not print).
#include "common.h"
#include "kernels.h"

namespace links {

namespace {

__device__ __forceinline__ int mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline double sqd2(double ax, double ay, double bx, double by) {
  double dx = ax - bx;
  double dy = ay - by;
  return dx * dx + dy * dy;
}

// 1/sqrt(x) for x > 0: hardware estimate (relative error below 2^-24 on gfx950)
// and one Newton step (below 2^-47; 4.2e-15 measured over 4M inputs spanning 600
// binades)
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  return y * fma(-hx * y, y, 1.5);
}

// Length drift of the links outside the solve order (only candidates with
// redundant links).  Returns true when one of them moved by more than thr.
__device__ bool drift_check(const SimArgs& A, int cand, int item, int D, int n, const double2* P, int bd, int tid,
                            double thr) {
  const int J = A.J;
  const size_t Bs = A.Bs;
  const uint32_t* adj = A.adj + (size_t)cand * J;
  const uint8_t* sj = A.slot_joint + item;
  const DyadF32* df = A.df + item;
  const double* x0 = A.x0 + (size_t)cand * J * 2;
  const int pivot = A.motor[2 * cand], tip = A.motor[2 * cand + 1];
  const uint32_t fixed = A.fixed[cand];
  for (int si = 0; si < n; ++si) {
    const int ji = sj[si * Bs];
    for (int sk = 0; sk < n; ++sk) {
      const int jk = sj[sk * Bs];
      if (jk <= ji || !((adj[ji] >> jk) & 1u)) continue;
      if ((ji == pivot && jk == tip) || (ji == tip && jk == pivot)) continue;
      bool parent_edge = false;
      if (si < D) {
        const uint32_t q = df[si * Bs].slots;
        parent_edge |= (int)(q & 0xFF) == sk || (int)((q >> 8) & 0xFF) == sk;
      }
      if (sk < D) {
        const uint32_t q = df[sk * Bs].slots;
        parent_edge |= (int)(q & 0xFF) == si || (int)((q >> 8) & 0xFF) == si;
      }
      if (parent_edge) continue;
      if (((fixed >> ji) & 1u) && ((fixed >> jk) & 1u)) continue;  // never moves
      const double L = sqrt(sqd2(x0[2 * ji], x0[2 * ji + 1], x0[2 * jk], x0[2 * jk + 1]));
      const double2 pi = P[si * bd + tid], pk = P[sk * bd + tid];
      const double now = sqrt(sqd2(pi.x, pi.y, pk.x, pk.y));
      if (fabs(now - L) > thr) return true;
    }
  }
  return false;
}

template <int DMAX, int SRC, bool EXACT>
__global__ void __launch_bounds__(256) sim64_kernel(SimArgs A) {
  extern __shared__ unsigned char smem[];
  const int bd = blockDim.x;
  const int tid = threadIdx.x;
  double2* P = reinterpret_cast<double2*>(smem);  // [nslot][bd]
  const int T = A.T;
  const int J = A.J;
  const int Bs = A.Bs;
  const int cnt_next = SRC == kFromEsc ? kCntEscNext : SRC == kFromPath ? kCntPathNext : kCntNext;
  const int cnt_items = SRC == kFromEsc ? kCntEsc : SRC == kFromPath ? kCntPath : kCntItems;

  int cand = -1, item = 0, t = 0, t_end = 0, D = 0, n = 0, out_slot = 0;
  int t_back = 0x7FFF;  // hand-over pass: step from which the candidate returns to FP32
  uint32_t sw[16];    // kFromPath: the current group of output positions (64 bytes)
#pragma unroll
  for (int i = 0; i < 16; ++i) sw[i] = 0u;
  int64_t row = -1;  // path row (kFromPath)
  bool redundant = false;
  const bool orient = A.branch != 0;  // sides fixed at the start (else continuity)
  uint32_t obits = 0u;                // starting side of each placed joint
  double px = 0, py = 0, vx = 0, vy = 0, deg_thr = 0, drift_thr = 0;
  bool exhausted = false;
  // Path chunks: a path-pass work item is one chunk of ck_len steps of a row; a
  // chunk after the first starts with the step before it, placed on the sides the
  // decision passes recorded there (forced) and not written.  The decision passes
  // record sb, the sides of the current step, every ck_len steps.
  // (the decision passes of FP64 precision and the hand-over pass record, every
  // path pass reads; with FP32 decisions the FP32 pass records the steps it
  // decides)
  constexpr bool REC = (SRC == kFromPerm && EXACT) || SRC == kFromEsc;
  constexpr bool CK = SRC == kFromPath;
  const bool chunked = CK && A.side_ck != nullptr;
  const int ckn = chunked ? A.ck_n : 1;
  uint32_t sb = 0u, fbits = 0u;
  bool forced = false;
  // per-entry constants of the lane's candidate, held in registers: S, Dm and
  // ra^2, rb^2 (EXACT) or Kc = (ra^2 - rb^2)/2 (fast)
  double cS[DMAX], cDm[DMAX], cA[DMAX], cB[DMAX];
  uint32_t cSl[DMAX];
#pragma unroll
  for (int s = 0; s < DMAX; ++s) {
    cS[s] = cDm[s] = cA[s] = cB[s] = 0.0;
    cSl[s] = 0u;
  }

  // Work is claimed in chunks of A.chunk list entries per atomic; the next chunk
  // is claimed ahead (after a refill's loads) and read when the current range
  // runs out.
  const int chunk = A.chunk;
  int cur_base = 0, cur_left = 0;   // entries claimed and not yet handed to lanes
  int pre_raw = 0, pre_req = 0;     // pending claim (return value meaningful in lane 0)
  bool pre_pending = false;
  const int nwaves = gridDim.x * (blockDim.x / kWave);
  bool no_more = false;             // a claim of this wave reached the end of the list
  for (;;) {
    uint64_t idle = __ballot(cand < 0);
    int nidle = __popcll(idle);
    if (nidle == kWave && exhausted) break;
    // idle lanes wait until enough of them can be refilled
    if (!exhausted && nidle > 0 && (nidle >= A.refill_min || nidle == kWave)) {
      const int items = A.counters[cnt_items] * ckn;
      int p = -1;
      for (int k = 0; k < 3 && nidle > 0; ++k) {
        if (cur_left == 0) {
          int base = 0, req = chunk;
          if (pre_pending) {
            base = __shfl(pre_raw, 0);
            req = pre_req;
            pre_pending = false;
          } else if (!no_more) {
            const int cur = __hip_atomic_load(&A.counters[cnt_next], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            req = min(chunk, max(nidle, max(items - cur, 0) / nwaves));
            if (__lane_id() == 0) base = atomicAdd(&A.counters[cnt_next], req);
            base = __shfl(base, 0);
          } else {
            break;
          }
          cur_base = base;
          cur_left = min(max(items - base, 0), req);
          if (base + req >= items) no_more = true;
        }
        const int m = min(nidle, cur_left);
        if (cand < 0 && p < 0) {
          const int r = mbcnt64(idle);
          if (r < m) p = cur_base + r;
        }
        cur_base += m;
        cur_left -= m;
        idle = __ballot(cand < 0 && p < 0);
        nidle = __popcll(idle);
      }
      exhausted = no_more && cur_left == 0 && !pre_pending;
      if (cand < 0) {
        if (p >= 0) {
          int it;
          int t0 = 0;
          bool from_x0 = true;
          if (SRC == kFromEsc) {
            const EscEntry e = A.esc[p];
            it = e.item;
            t0 = e.t;
            from_x0 = e.from_x0 != 0;
          } else if (SRC == kFromPath) {
            it = A.path_list[chunked ? p / ckn : p];
          } else {
            it = p;
          }
          const int c = A.perm[it];
          item = it;
          t = t0;
          t_back = 0x7FFF;
          t_end = T;
          bool take = true;
          if (SRC == kFromPath) {
            row = A.write_all ? (int64_t)c : (int64_t)A.path_row[c];
            const int fs = A.fail_step[c];
            if (fs >= 0) t_end = fs;  // the path exists up to the failing step
            forced = false;
            if (chunked) {
              const int kc = p % ckn, t0c = kc * kPathChunk;
              t_end = min(t_end, t0c + kPathChunk);
              if (kc > 0) {
                if (t0c < t_end) {
                  forced = true;
                  fbits = A.side_ck[(size_t)c * ckn + kc];
                  t = t0c - 1;
                } else {
                  t_end = 0;  // the row ends before this chunk
                }
              }
            }
            take = row >= 0 && t < t_end && t_end > 0;
          }
          if (take) {
            const CandMeta m = A.meta[it];
            cand = (SRC == kFromPath && (m.flags & kFlagNoPath)) ? -1 : c;
            D = m.D;
            n = m.n;
            out_slot = m.out_slot;
            redundant = (m.flags & kFlagRedundant) != 0;
            // drift checks need FP64 lengths, so those candidates stay
            if (SRC == kFromEsc && A.deesc > 0 && !redundant) t_back = t + A.deesc;
            const CandF64 f = A.cd[it];
            px = f.px;
            py = f.py;
            vx = f.vx;
            vy = f.vy;
            deg_thr = f.deg_thr;
            drift_thr = f.drift_thr;
            obits = (uint32_t)f.side;
#pragma unroll
            for (int s = 0; s < DMAX; ++s) {
              if (s < D) {
                const DyadF64 q = A.dd[(size_t)s * Bs + it];
                cS[s] = q.S;
                cDm[s] = q.Dm;
                if (EXACT) {
                  cA[s] = q.ra2;
                  cB[s] = q.rb2;
                } else {
                  cA[s] = 0.5 * (q.ra2 - q.rb2);
                }
                cSl[s] = A.df[(size_t)s * Bs + it].slots;
              }
            }
            const double2* x0 = reinterpret_cast<const double2*>(A.x0 + (size_t)c * J * 2);
            const float2* dump = SRC == kFromEsc ? A.esc_pos + (size_t)it * J : nullptr;
            // initial positions, four slots at a time: the slot -> joint maps of
            // the group, then its positions, each set of loads issued together
            constexpr int NMAX = DMAX + 2;  // joints per candidate at most (J of this template)
            constexpr int G = 4;
#pragma unroll
            for (int g = 0; g < NMAX; g += G) {
              int jq[G];
#pragma unroll
              for (int k = 0; k < G; ++k) {
                const int sl = g + k;
                jq[k] = 0;
                if (sl < n && (sl > D || from_x0)) jq[k] = A.slot_joint[(size_t)sl * Bs + it];
              }
              double qx[G], qy[G];
#pragma unroll
              for (int k = 0; k < G; ++k) {
                const int sl = g + k;
                qx[k] = 0.0;
                qy[k] = 0.0;
                if (sl < n) {
                  if (sl > D || from_x0) {  // fixed joints, or reference positions at t = 0
                    const double2 q = x0[jq[k]];
                    qx[k] = q.x;
                    qy[k] = q.y;
                  } else {
                    const float2 q = dump[sl];
                    qx[k] = (double)q.x;
                    qy[k] = (double)q.y;
                  }
                }
              }
#pragma unroll
              for (int k = 0; k < G; ++k)
                if (g + k < n) P[(g + k) * bd + tid] = make_double2(qx[k], qy[k]);
            }
          }
        }
      }
      // claim the next chunk ahead, after this refill's loads; guided size: the
      // waves' share of what remains after the current range, at most chunk
      if (!pre_pending && !no_more && cur_left < chunk) {
        const int share = max(items - (cur_base + cur_left), 0) / nwaves;
        pre_req = min(chunk, max(share, max(A.refill_min, 1)));
        if (__lane_id() == 0) pre_raw = atomicAdd(&A.counters[cnt_next], pre_req);
        pre_pending = true;
      }
    }
    if (cand >= 0) {
      const double2 cs = A.cs64[t];
      const double ct = cs.x, st = cs.y;
      if (EXACT)
        P[D * bd + tid] = make_double2(px + (ct * vx - st * vy), py + (st * vx + ct * vy));
      else
        P[D * bd + tid] = make_double2(fma(ct, vx, fma(-st, vy, px)), fma(st, vx, fma(ct, vy, py)));
      int fail = 0;
      sb = 0u;
#pragma unroll
      for (int s = 0; s < DMAX; ++s) {
        if (s < D && fail == 0) {
          const uint32_t sl = cSl[s];
          const int a = sl & 0xFF, b = (sl >> 8) & 0xFF;
          const double2 pa = P[a * bd + tid];
          const double2 pb = P[b * bd + tid];
          const double2 pr = P[s * bd + tid];
          const double dx = pb.x - pa.x;
          const double dy = pb.y - pa.y;
          if (EXACT) {
            const double d2 = dx * dx + dy * dy;
            if (d2 <= deg_thr) {
              fail = 2;
            } else {
              const double K = (cS[s] - d2) * (d2 - cDm[s]);
              if (K < 0.0) {
                fail = 1;
              } else {
                const double d = sqrt(d2);
                const double h = sqrt(K) / (2.0 * d);
                const double along = (d2 + cA[s] - cB[s]) / (2.0 * d);
                const double bx = pa.x + (along / d) * dx;
                const double by = pa.y + (along / d) * dy;
                const double ox = -(h / d) * dy;
                const double oy = (h / d) * dx;
                const double cpx = bx + ox, cpy = by + oy;
                const double cmx = bx - ox, cmy = by - oy;
                const double dp2 = (pr.x - cpx) * (pr.x - cpx) + (pr.y - cpy) * (pr.y - cpy);
                const double dm2 = (pr.x - cmx) * (pr.x - cmx) + (pr.y - cmy) * (pr.y - cmy);
                const bool left = (orient || forced) ? (((forced ? fbits : obits) >> s) & 1u) != 0u : dp2 <= dm2;
                if (REC) sb |= (left ? 1u : 0u) << s;
                P[s * bd + tid] = left ? make_double2(cpx, cpy) : make_double2(cmx, cmy);
              }
            }
          } else {
            const double d2 = fma(dy, dy, dx * dx);
            const double K = (cS[s] - d2) * (d2 - cDm[s]);
            if (d2 <= deg_thr) {
              fail = 2;
            } else if (K < 0.0) {
              fail = 1;
            } else {
              const double rd = rsqrt_nr(d2);
              const double inv = rd * rd;
              const double Kp = fmax(K, 1e-300);
              const double sK = Kp * rsqrt_nr(Kp);
              const double al = fma(cA[s], inv, 0.5);
              const double be = sK * (0.5 * inv);
              const double bx = fma(al, dx, pa.x), by = fma(al, dy, pa.y);
              const double ox = -be * dy, oy = be * dx;
              const double sg = fma(pr.x - bx, ox, (pr.y - by) * oy);
              const bool left = (orient || forced) ? (((forced ? fbits : obits) >> s) & 1u) != 0u : sg >= 0.0;
              if (REC) sb |= (left ? 1u : 0u) << s;
              const double sgn = left ? 1.0 : -1.0;
              P[s * bd + tid] = make_double2(fma(sgn, ox, bx), fma(sgn, oy, by));
            }
          }
        }
      }
      if (fail == 0 && redundant && drift_check(A, cand, item, D, n, P, bd, tid, drift_thr)) fail = 3;
      if (REC && A.side_ck != nullptr && fail == 0 && t + 1 < T && ((t + 1) & (kPathChunk - 1)) == 0)
        A.side_ck[(size_t)cand * A.ck_n + (t + 1) / kPathChunk] = sb;
      bool done = false;
      if (CK && forced) {
        // the step before the chunk: its positions only
        forced = false;
        if (fail != 0) {
          // (possible only within rounding of a threshold) the chunk's row stays NaN
          const double nan = __builtin_nan("");
          for (int tt = t + 1; tt < t_end; ++tt) {
            if (A.path_f64)
              reinterpret_cast<double2*>(A.path)[row * T + tt] = make_double2(nan, nan);
            else
              reinterpret_cast<float2*>(A.path)[row * T + tt] = make_float2((float)nan, (float)nan);
          }
          done = true;
        } else {
          ++t;
        }
      } else if (SRC == kFromPath && EXACT && DMAX > 11) {
        // (the correctly rounded sequence above 13 joints needs every register for
        // its arithmetic: a store per step)
        double2 po = P[out_slot * bd + tid];
        if (fail != 0) po = make_double2(__builtin_nan(""), __builtin_nan(""));
        const int t_stop = fail != 0 ? t_end : t + 1;
        // a failure here (possible only within rounding of a threshold) leaves the
        // rest of the row NaN
        for (int tt = t; tt < t_stop; ++tt) {
          if (A.path_f64)
            reinterpret_cast<double2*>(A.path)[row * T + tt] = po;
          else
            reinterpret_cast<float2*>(A.path)[row * T + tt] = make_float2((float)po.x, (float)po.y);
        }
        if (fail != 0 || ++t >= t_end) done = true;
      } else if (SRC == kFromPath) {
        // the row is written 64 bytes at a time: the last K steps' positions staged
        // in registers (K = 8 for f32 paths, 4 for f64) and stored together as four
        // 16-byte pieces, so each lane's row reaches memory in whole 64-byte
        // segments rather than one 8-byte store per step
        const int K = A.path_f64 ? 4 : 8;
        const int k = t & (K - 1);
        const int t_first = t - k;
        int staged = k;  // entries of the group already staged (steps t_first .. t - 1)
        if (fail == 0) {
          const double2 po = P[out_slot * bd + tid];
          // the entry's dwords: 4 for an f64 position, 2 for an f32 one
          if (A.path_f64) {
            const uint32_t v[4] = {(uint32_t)__double2loint(po.x), (uint32_t)__double2hiint(po.x),
                                   (uint32_t)__double2loint(po.y), (uint32_t)__double2hiint(po.y)};
#pragma unroll
            for (int i = 0; i < 16; ++i) sw[i] = i / 4 == k ? v[i % 4] : sw[i];
          } else {
            const uint32_t v[2] = {__float_as_uint((float)po.x), __float_as_uint((float)po.y)};
#pragma unroll
            for (int i = 0; i < 16; ++i) sw[i] = i / 2 == k ? v[i % 2] : sw[i];
          }
          staged = k + 1;
        }
        const bool flush = fail != 0 || staged == K || t + 1 >= t_end;
        if (flush && staged > 0) {
          if (staged == K && (A.path_f64 || (T & 1) == 0)) {
            // a whole group: four 16-byte stores (16-byte aligned: t_first is a
            // multiple of K and rows of an even T start on 16 bytes)
            uint4* dst = reinterpret_cast<uint4*>(reinterpret_cast<char*>(A.path) +
                                                  (size_t)(row * T + t_first) * (A.path_f64 ? 16 : 8));
#pragma unroll
            for (int j = 0; j < 4; ++j) dst[j] = make_uint4(sw[4 * j], sw[4 * j + 1], sw[4 * j + 2], sw[4 * j + 3]);
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              if (j < staged) {
                if (A.path_f64) {
                  if (j < 4)
                    reinterpret_cast<double2*>(A.path)[row * T + t_first + j] = make_double2(
                        __hiloint2double(sw[4 * j + 1], sw[4 * j]), __hiloint2double(sw[4 * j + 3], sw[4 * j + 2]));
                } else {
                  reinterpret_cast<float2*>(A.path)[row * T + t_first + j] =
                      make_float2(__uint_as_float(sw[2 * j]), __uint_as_float(sw[2 * j + 1]));
                }
              }
            }
          }
        }
        if (fail != 0) {
          // a failure here (possible only within rounding of a threshold) leaves the
          // rest of the row NaN
          const double nan = __builtin_nan("");
          for (int tt = t; tt < t_end; ++tt) {
            if (A.path_f64)
              reinterpret_cast<double2*>(A.path)[row * T + tt] = make_double2(nan, nan);
            else
              reinterpret_cast<float2*>(A.path)[row * T + tt] = make_float2((float)nan, (float)nan);
          }
        }
        if (fail != 0 || ++t >= t_end) done = true;
      } else if (fail != 0) {
        A.status[cand] = (uint8_t)fail;
        A.fail_step[cand] = (int16_t)t;
        if (SRC == kFromPerm && A.esc_step) A.esc_step[cand] = -1;  // FP64 throughout: never handed over
        done = true;
      } else if (++t == T) {
        A.status[cand] = 0;
        A.fail_step[cand] = -1;
        if (SRC == kFromPerm && A.esc_step) A.esc_step[cand] = -1;
        done = true;
      } else if (SRC == kFromEsc && t >= t_back) {
        // decided in FP64 up to here: back to FP32 from step t with these positions
        const int r = atomicAdd(&A.counters[kCntRes], 1);
        EscEntry e;
        e.item = item;
        e.t = (int16_t)t;
        e.from_x0 = 0;
        e.pad = 0;
        A.res[r] = e;
        float2* dump = A.res_pos + (size_t)r * J;
        for (int sl = 0; sl < n; ++sl) {
          const double2 q = P[sl * bd + tid];
          dump[sl] = make_float2((float)q.x, (float)q.y);
        }
        done = true;
      }
      if (done) cand = -1;
    }
  }
}

template <int DMAX, int SRC, bool EXACT>
void launch_one(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  const int bd = cfg.waves * kWave;
  const size_t lds = (size_t)a.nslot * bd * sizeof(double2);
  hipLaunchKernelGGL((sim64_kernel<DMAX, SRC, EXACT>), dim3(cfg.grid), dim3(bd), lds, st, a);
}

template <int SRC, bool EXACT>
hipError_t dispatch(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  switch (sim32_dmax(a.J)) {
    case 5: launch_one<5, SRC, EXACT>(a, cfg, st); break;
    case 11: launch_one<11, SRC, EXACT>(a, cfg, st); break;
    case 18: launch_one<18, SRC, EXACT>(a, cfg, st); break;
    default: launch_one<30, SRC, EXACT>(a, cfg, st); break;
  }
  return hipGetLastError();
}

template <int DMAX, int SRC, bool EXACT>
int occ(int waves, int lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sim64_kernel<DMAX, SRC, EXACT>, waves * kWave, lds) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <int SRC, bool EXACT>
int occ_for(int J, int waves, int lds) {
  switch (sim32_dmax(J)) {
    case 5: return occ<5, SRC, EXACT>(waves, lds);
    case 11: return occ<11, SRC, EXACT>(waves, lds);
    case 18: return occ<18, SRC, EXACT>(waves, lds);
    default: return occ<30, SRC, EXACT>(waves, lds);
  }
}

// ---- the same passes, parallel in time.
//
// A segment of W lanes (within one 16-lane DPP row) holds one candidate, and lane r of the
// segment computes step t0 - 1 + r.  Lane 0, the provider, recomputes the last step
// already decided (or holds the starting positions), so that every other lane finds
// its candidate's previous positions in its left neighbour.  Every dyad is placed on
// an assumed side of its parents' line (one orientation bit per dyad, first taken
// from the starting positions); each computing lane then applies the continuity
// rule against its neighbour's position.  The first lane, in step order, where the
// rule picks the other side, a placement fails or a link drifts ends the pass for
// the segment.  Up to that lane every choice was the rule's, so the lanes computed
// exactly what the step-by-step recurrence computes (a position depends on the
// earlier steps only through the side chosen).  A failure is the candidate's
// outcome at that step; a side change flips the dyad's bit and the segment
// restarts at that step, where the rule now agrees with the bit up to that dyad (so
// at most D restarts happen at one step).

// the value held by lane - 1 of the same 16-lane row (lane 0 of a row gets 0)
__device__ __forceinline__ double row_prev(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x111, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x111, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

enum : int { kEvNone = 0, kEvLock = 1, kEvDegenerate = 2, kEvDrift = 3, kEvSide = 4 };

// per-entry constants of a segment's candidate, in LDS: S, Dm and ra^2, rb^2
// (EXACT) or Kc = (ra^2 - rb^2)/2 in A (fast)
struct DyadC {
  double S, Dm, A, B;
};

// LDS of the parallel pass: positions [nslot][bd] and, per segment, DMAX entries
// of constants and their parent slots
template <int DMAX, int W>
__host__ __device__ constexpr size_t par_lds_bytes(int nslot, int bd) {
  return (size_t)nslot * bd * sizeof(double2) + (size_t)(bd / W) * DMAX * (sizeof(DyadC) + sizeof(uint32_t));
}

template <int DMAX, int SRC, bool EXACT, int W>
__global__ void __launch_bounds__(256) simpar64_kernel(SimArgs A) {
  static_assert(W == 4 || W == 8 || W == 16, "segments lie within 16-lane DPP rows");
  constexpr int NQ = 32 / W;  // entries and slots each lane loads at a refill
  constexpr uint32_t WMASK = (1u << W) - 1u;
  extern __shared__ unsigned char smem[];
  const int bd = blockDim.x;
  const int tid = threadIdx.x;
  double2* P = reinterpret_cast<double2*>(smem);  // [nslot][bd]
  const int T = A.T;
  const int J = A.J;
  const int Bs = A.Bs;
  const int lane = __lane_id();
  const int r = lane & (W - 1);    // position in the segment; 0 is the provider
  const int seg0 = lane & ~(W - 1);
  const int segb = tid / W;        // segment of the workgroup
  DyadC* C = reinterpret_cast<DyadC*>(smem + (size_t)A.nslot * bd * sizeof(double2)) + segb * DMAX;
  uint32_t* SL = reinterpret_cast<uint32_t*>(smem + (size_t)A.nslot * bd * sizeof(double2) +
                                             (size_t)(bd / W) * DMAX * sizeof(DyadC)) + segb * DMAX;
  const int cnt_next = SRC == kFromEsc ? kCntEscNext : SRC == kFromPath ? kCntPathNext : kCntNext;
  const int cnt_items = SRC == kFromEsc ? kCntEsc : SRC == kFromPath ? kCntPath : kCntItems;

  // segment state (the same in every lane of a segment)
  int cand = -1, item = 0, t0 = 0, t_end = 0, D = 0, n = 0, out_slot = 0, restarts = 0;
  int64_t row = -1;
  bool redundant = false;
  const bool orient = A.branch != 0;  // sides fixed at the start (else continuity)
  uint32_t obits = 0u;
  bool fresh = false;             // the provider holds the starting positions
  uint32_t ori = 0u;              // side of every dyad for the computing lanes (bit set: left of a->b)
  uint32_t ori_prov = 0u;         // the sides in force at the provider's step
  double px = 0, py = 0, vx = 0, vy = 0, deg_thr = 0, drift_thr = 0;
  int dmax_w = 0;                 // largest solve order among the wave's segments

  const int chunk = A.chunk;
  int cur_base = 0, cur_left = 0;
  bool no_more = false, exhausted = false;
  const int nwaves = gridDim.x * (bd / kWave);
  const int items = A.counters[cnt_items];
  for (;;) {
    // ---- segments without a candidate take the next list entries, in lane order
    const uint64_t idle = __ballot(cand < 0 && r == 0);
    const int nidle = __popcll(idle);
    if (nidle == kWave / W && exhausted) break;
    if (!exhausted && nidle > 0) {
      const int rank = __popcll(idle & ((1ull << seg0) - 1ull));  // idle segments before this one
      int p = -1, given = 0;
      for (int k = 0; k < 3 && given < nidle; ++k) {
        if (cur_left == 0) {
          if (no_more) break;
          const int cur = __hip_atomic_load(&A.counters[cnt_next], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const int req = min(chunk, max(nidle - given, max(items - cur, 0) / nwaves));
          int base = 0;
          if (lane == 0) base = atomicAdd(&A.counters[cnt_next], req);
          base = __shfl(base, 0);
          cur_base = base;
          cur_left = min(max(items - base, 0), req);
          if (base + req >= items) no_more = true;
        }
        const int m = min(nidle - given, cur_left);
        if (cand < 0 && rank >= given && rank < given + m) p = cur_base + (rank - given);
        cur_base += m;
        cur_left -= m;
        given += m;
      }
      exhausted = no_more && cur_left == 0;
      bool fill = false;  // this segment takes a candidate now
      double2 vs[NQ];
#pragma unroll
      for (int k = 0; k < NQ; ++k) vs[k] = make_double2(0.0, 0.0);
      if (p >= 0) {
        // list entry, then everything the item addresses, each level's loads issued
        // together; the segment's lanes share the per-entry and per-slot loads
        int it, ts = 0;
        bool from_x0 = true;
        if (SRC == kFromEsc) {
          const EscEntry e = A.esc[p];
          it = e.item;
          ts = e.t;
          from_x0 = e.from_x0 != 0;
        } else if (SRC == kFromPath) {
          it = A.path_list[p];
        } else {
          it = p;
        }
        const int c = A.perm[it];
        const CandMeta m = A.meta[it];
        const CandF64 f = A.cd[it];
        int fs = -1;
        if (SRC == kFromPath) fs = A.fail_step[c];
        const int mD = m.D, mn = m.n;
        // lane r: entries and slots r + k W
        DyadF64 q[NQ];
        uint32_t lq[NQ];
        int jq[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
          const int e = min(r + k * W, max(mD - 1, 0));
          q[k] = A.dd[(size_t)e * Bs + it];
          lq[k] = A.df[(size_t)e * Bs + it].slots;
          jq[k] = A.slot_joint[(size_t)min(r + k * W, mn - 1) * Bs + it];
        }
        const double2* x0 = reinterpret_cast<const double2*>(A.x0 + (size_t)c * J * 2);
        double2 vq[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) vq[k] = x0[jq[k]];
        if (SRC == kFromEsc && !from_x0) {
          const float2* dump = A.esc_pos + (size_t)it * J;
#pragma unroll
          for (int k = 0; k < NQ; ++k) {
            const float2 w = dump[min(r + k * W, mn - 1)];
            if (r + k * W <= mD) vq[k] = make_double2((double)w.x, (double)w.y);
          }
        }
        item = it;
        t_end = T;
        bool take = true;
        if (SRC == kFromPath) {
          row = A.write_all ? (int64_t)c : (int64_t)A.path_row[c];
          if (fs >= 0) t_end = fs;  // the path exists up to the failing step
          take = row >= 0 && t_end > 0 && !(m.flags & kFlagNoPath);
        }
        if (take) {
          cand = c;
          D = mD;
          n = mn;
          out_slot = m.out_slot;
          redundant = (m.flags & kFlagRedundant) != 0;
          px = f.px;
          py = f.py;
          vx = f.vx;
          vy = f.vy;
          deg_thr = f.deg_thr;
          drift_thr = f.drift_thr;
          obits = (uint32_t)f.side;
          t0 = ts;
          fresh = true;
          restarts = 0;
          fill = true;
#pragma unroll
          for (int k = 0; k < NQ; ++k) {
            const int se = r + k * W;
            if (se < D) {
              C[se] = DyadC{q[k].S, q[k].Dm, EXACT ? q[k].ra2 : 0.5 * (q[k].ra2 - q[k].rb2), q[k].rb2};
              SL[se] = lq[k];
            }
            vs[k] = vq[k];
          }
        }
      }
      // starting positions of slots kk + k W, broadcast from lane kk of the
      // segment; every lane writes its own column (conflict-free)
      for (int kk = 0; kk < W; ++kk) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
          const double2 u = make_double2(__shfl(vs[k].x, seg0 + kk), __shfl(vs[k].y, seg0 + kk));
          if (fill && kk + k * W < n) P[(kk + k * W) * bd + tid] = u;
        }
      }
      // the segment's LDS writes are complete before any lane reads them (LDS
      // operations of a wave complete in order; only the compiler is held back)
      __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
      asm volatile("" ::: "memory");
      // first guess of the sides: those of the starting positions (lane r: dyads r + k W)
      uint32_t og = 0u;
#pragma unroll
      for (int k = 0; k < NQ; ++k) {
        const int se = r + k * W;
        bool g = false;
        if (fill && se < D) {
          const uint32_t sl = SL[se];
          const double2 pa = P[(sl & 0xFF) * bd + tid], pb = P[((sl >> 8) & 0xFF) * bd + tid], pk = P[se * bd + tid];
          g = (pb.x - pa.x) * (pk.y - pa.y) - (pb.y - pa.y) * (pk.x - pa.x) >= 0.0;
        }
        og |= (uint32_t)((__ballot(g) >> seg0) & WMASK) << (k * W);
      }
      if (fill) {
        ori = orient ? obits : og;
        ori_prov = ori;
      }
      // largest solve order among the wave's segments (bounds the dyad loop)
      int dm = cand >= 0 ? D : 0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) dm = max(dm, __shfl_xor(dm, off));
      dmax_w = dm;
    }
    if (__ballot(cand >= 0) == 0ull) continue;

    // ---- one pass: lane r computes step t
    const int t = t0 - 1 + r;
    const bool comp = cand >= 0 && t < t_end && !(r == 0 && fresh);
    const uint32_t side = r == 0 ? ori_prov : ori;
    if (comp) {
      const double2 cs = A.cs64[t];
      const double ct = cs.x, st = cs.y;
      if (EXACT)
        P[D * bd + tid] = make_double2(px + (ct * vx - st * vy), py + (st * vx + ct * vy));
      else
        P[D * bd + tid] = make_double2(fma(ct, vx, fma(-st, vy, px)), fma(st, vx, fma(ct, vy, py)));
    }
    int ev = kEvNone, ev_s = 0;
#pragma unroll
    for (int s = 0; s < DMAX; ++s) {
      if (s < dmax_w) {
        const bool act = comp && s < D && ev == kEvNone;
        double2 val = P[s * bd + tid];
        // EXACT: both intersections; fast: base point and offset
        double rx0 = 0, ry0 = 0, rx1 = 0, ry1 = 0;
        bool placed = false;
        if (act) {
          const uint32_t sl = SL[s];
          const DyadC q = C[s];
          const int a = sl & 0xFF, b = (sl >> 8) & 0xFF;
          const double2 pa = P[a * bd + tid];
          const double2 pb = P[b * bd + tid];
          const double dx = pb.x - pa.x;
          const double dy = pb.y - pa.y;
          const bool left = (side >> s) & 1u;
          if (EXACT) {
            const double d2 = dx * dx + dy * dy;
            if (d2 <= deg_thr) {
              ev = kEvDegenerate;
            } else {
              const double K = (q.S - d2) * (d2 - q.Dm);
              if (K < 0.0) {
                ev = kEvLock;
              } else {
                const double d = sqrt(d2);
                const double h = sqrt(K) / (2.0 * d);
                const double along = (d2 + q.A - q.B) / (2.0 * d);
                const double bx = pa.x + (along / d) * dx;
                const double by = pa.y + (along / d) * dy;
                const double ox = -(h / d) * dy;
                const double oy = (h / d) * dx;
                rx0 = bx + ox;
                ry0 = by + oy;
                rx1 = bx - ox;
                ry1 = by - oy;
                val = left ? make_double2(rx0, ry0) : make_double2(rx1, ry1);
                placed = true;
              }
            }
          } else {
            const double d2 = fma(dy, dy, dx * dx);
            const double K = (q.S - d2) * (d2 - q.Dm);
            if (d2 <= deg_thr) {
              ev = kEvDegenerate;
            } else if (K < 0.0) {
              ev = kEvLock;
            } else {
              const double rd = rsqrt_nr(d2);
              const double inv = rd * rd;
              const double Kp = fmax(K, 1e-300);
              const double sK = Kp * rsqrt_nr(Kp);
              const double al = fma(q.A, inv, 0.5);
              const double be = sK * (0.5 * inv);
              rx0 = fma(al, dx, pa.x);
              ry0 = fma(al, dy, pa.y);
              rx1 = -be * dy;
              ry1 = be * dx;
              const double sgn = left ? 1.0 : -1.0;
              val = make_double2(fma(sgn, rx1, rx0), fma(sgn, ry1, ry0));
              placed = true;
            }
          }
          if (placed) P[s * bd + tid] = val;
        }
        // the previous step's position of this joint, from the left neighbour
        const double qx = row_prev(val.x), qy = row_prev(val.y);
        if (placed && r > 0 && !orient) {
          bool rule_left;
          if (EXACT) {
            const double dp2 = (qx - rx0) * (qx - rx0) + (qy - ry0) * (qy - ry0);
            const double dm2 = (qx - rx1) * (qx - rx1) + (qy - ry1) * (qy - ry1);
            rule_left = dp2 <= dm2;
          } else {
            rule_left = fma(qx - rx0, rx1, (qy - ry0) * ry1) >= 0.0;
          }
          if (rule_left != (((side >> s) & 1u) != 0u)) {
            ev = kEvSide;
            ev_s = s;
          }
        }
      }
    }
    if (comp && r > 0 && ev == kEvNone && redundant && drift_check(A, cand, item, D, n, P, bd, tid, drift_thr))
      ev = kEvDrift;

    // ---- the segment's first event, in step order
    const uint64_t evb = __ballot(comp && r > 0 && ev != kEvNone);
    const uint32_t segm = (uint32_t)(evb >> seg0) & WMASK;
    const int f = segm ? __ffs(segm) - 1 : W;
    const int info = __shfl(ev | (ev_s << 8), seg0 + (f < W ? f : 0));
    const int kind = f < W ? (info & 0xFF) : kEvNone;
    // the sides of each decided step that ends a chunk of a path row (lanes before
    // the segment's first event), for the chunked path pass
    if (SRC != kFromPath && A.side_ck != nullptr && comp && r > 0 && r < f && t + 1 < T &&
        ((t + 1) & (kPathChunk - 1)) == 0)
      A.side_ck[(size_t)cand * A.ck_n + (t + 1) / kPathChunk] = side;
    if (SRC == kFromPath && comp && r > 0 && r < f) {
      const double2 po = P[out_slot * bd + tid];
      if (A.path_f64)
        reinterpret_cast<double2*>(A.path)[row * T + t] = po;
      else
        reinterpret_cast<float2*>(A.path)[row * T + t] = make_float2((float)po.x, (float)po.y);
    }
    if (cand >= 0) {
      bool done = false;
      const int te = t0 - 1 + f;  // step of the event
      if (kind == kEvNone) {
        const int next = t0 + (W - 1);
        if (next >= t_end) {
          if (SRC != kFromPath && r == 0) {
            A.status[cand] = 0;
            A.fail_step[cand] = -1;
            if (SRC == kFromPerm && A.esc_step) A.esc_step[cand] = -1;
          }
          done = true;
        } else {
          t0 = next;
          ori_prov = ori;
          fresh = false;
          restarts = 0;
        }
      } else if (kind == kEvSide) {
        // the provider of the restarted pass is the step before the change
        if (f >= 2) {
          ori_prov = ori;
          fresh = false;
          restarts = 0;
        }
        ori ^= 1u << (info >> 8);
        t0 = te;
        if (++restarts > D + 1) {
          // cannot happen (each restart at one step moves the first change to a
          // later dyad); the candidate is left without a final status
          if (SRC != kFromPath && r == 0) A.status[cand] = kPending;
          done = true;
        }
      } else {
        if (SRC == kFromPath) {
          // a failure here (possible only within rounding of a threshold) leaves the
          // rest of the row NaN
          const double nan = __builtin_nan("");
          for (int tt = te + r; tt < t_end; tt += W) {
            if (A.path_f64)
              reinterpret_cast<double2*>(A.path)[row * T + tt] = make_double2(nan, nan);
            else
              reinterpret_cast<float2*>(A.path)[row * T + tt] = make_float2((float)nan, (float)nan);
          }
        } else if (r == 0) {
          A.status[cand] = (uint8_t)kind;
          A.fail_step[cand] = (int16_t)te;
          if (SRC == kFromPerm && A.esc_step) A.esc_step[cand] = -1;
        }
        done = true;
      }
      if (done) cand = -1;
    }
  }
}

template <int DMAX, int SRC, bool EXACT, int W>
void launch_par_w(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  const int bd = cfg.waves * kWave;
  const size_t lds = par_lds_bytes<DMAX, W>(a.nslot, bd);
  hipLaunchKernelGGL((simpar64_kernel<DMAX, SRC, EXACT, W>), dim3(cfg.grid), dim3(bd), lds, st, a);
}

template <int DMAX, int SRC, bool EXACT>
void launch_par_one(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  if constexpr (SRC == kFromEsc) {
    if (cfg.seg == 8) return launch_par_w<DMAX, SRC, EXACT, 8>(a, cfg, st);
    if (cfg.seg == 4) return launch_par_w<DMAX, SRC, EXACT, 4>(a, cfg, st);
  }
  launch_par_w<DMAX, SRC, EXACT, 16>(a, cfg, st);
}

template <int SRC, bool EXACT>
hipError_t dispatch_par(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  switch (sim32_dmax(a.J)) {
    case 5: launch_par_one<5, SRC, EXACT>(a, cfg, st); break;
    case 11: launch_par_one<11, SRC, EXACT>(a, cfg, st); break;
    case 18: launch_par_one<18, SRC, EXACT>(a, cfg, st); break;
    default: launch_par_one<30, SRC, EXACT>(a, cfg, st); break;
  }
  return hipGetLastError();
}

template <int DMAX, int SRC, bool EXACT, int W>
int occ_par_w(int J, int waves) {
  const int lds = (int)par_lds_bytes<DMAX, W>(J, waves * kWave);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, simpar64_kernel<DMAX, SRC, EXACT, W>, waves * kWave, lds) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <int DMAX, int SRC, bool EXACT>
int occ_par(int J, int waves, int seg) {
  if constexpr (SRC == kFromEsc) {
    if (seg == 8) return occ_par_w<DMAX, SRC, EXACT, 8>(J, waves);
    if (seg == 4) return occ_par_w<DMAX, SRC, EXACT, 4>(J, waves);
  }
  return occ_par_w<DMAX, SRC, EXACT, 16>(J, waves);
}

template <int SRC, bool EXACT>
int occ_par_for(int J, int waves, int seg) {
  switch (sim32_dmax(J)) {
    case 5: return occ_par<5, SRC, EXACT>(J, waves, seg);
    case 11: return occ_par<11, SRC, EXACT>(J, waves, seg);
    case 18: return occ_par<18, SRC, EXACT>(J, waves, seg);
    default: return occ_par<30, SRC, EXACT>(J, waves, seg);
  }
}

}  // namespace

int sim64_lds_bytes(int nslot, int waves) { return nslot * waves * kWave * (int)sizeof(double2); }

hipError_t launch_sim64(const SimArgs& a, int source, bool exact, const LaunchCfg& cfg, hipStream_t st) {
  if (exact) {
    switch (source) {
      case kFromEsc: return dispatch<kFromEsc, true>(a, cfg, st);
      case kFromPath: return dispatch<kFromPath, true>(a, cfg, st);
      default: return dispatch<kFromPerm, true>(a, cfg, st);
    }
  }
  switch (source) {
    case kFromEsc: return dispatch<kFromEsc, false>(a, cfg, st);
    case kFromPath: return dispatch<kFromPath, false>(a, cfg, st);
    default: return dispatch<kFromPerm, false>(a, cfg, st);
  }
}

int sim64_blocks_per_cu(int J, int source, bool exact, int waves, int lds) {
  if (exact) {
    switch (source) {
      case kFromEsc: return occ_for<kFromEsc, true>(J, waves, lds);
      case kFromPath: return occ_for<kFromPath, true>(J, waves, lds);
      default: return occ_for<kFromPerm, true>(J, waves, lds);
    }
  }
  switch (source) {
    case kFromEsc: return occ_for<kFromEsc, false>(J, waves, lds);
    case kFromPath: return occ_for<kFromPath, false>(J, waves, lds);
    default: return occ_for<kFromPerm, false>(J, waves, lds);
  }
}

hipError_t launch_sim64_par(const SimArgs& a, int source, bool exact, const LaunchCfg& cfg, hipStream_t st) {
  if (exact) {
    switch (source) {
      case kFromEsc: return dispatch_par<kFromEsc, true>(a, cfg, st);
      case kFromPath: return dispatch_par<kFromPath, true>(a, cfg, st);
      default: return dispatch_par<kFromPerm, true>(a, cfg, st);
    }
  }
  switch (source) {
    case kFromEsc: return dispatch_par<kFromEsc, false>(a, cfg, st);
    case kFromPath: return dispatch_par<kFromPath, false>(a, cfg, st);
    default: return dispatch_par<kFromPerm, false>(a, cfg, st);
  }
}

int sim64_par_blocks_per_cu(int J, int source, bool exact, int waves, int seg) {
  if (exact) {
    switch (source) {
      case kFromEsc: return occ_par_for<kFromEsc, true>(J, waves, seg);
      case kFromPath: return occ_par_for<kFromPath, true>(J, waves, seg);
      default: return occ_par_for<kFromPerm, true>(J, waves, seg);
    }
  }
  switch (source) {
    case kFromEsc: return occ_par_for<kFromEsc, false>(J, waves, seg);
    case kFromPath: return occ_par_for<kFromPath, false>(J, waves, seg);
    default: return occ_par_for<kFromPerm, false>(J, waves, seg);
  }
}

}  // namespace links
