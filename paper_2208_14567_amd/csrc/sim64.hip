// sim64.hip -- FP64 simulation pass.  Runs either every pending candidate from
// t = 0 (plain FP64 precision) or the candidates the FP32 pass handed over, from
// the step at which they were handed over.
//
// The arithmetic of one step is written as the sequence of correctly rounded
// double operations below, with no contraction into fused multiply-adds (the
// library is built with -ffp-contract=off):
//   tip   = pivot + (cos t * v_x - sin t * v_y, sin t * v_x + cos t * v_y)
//   d^2   = dx*dx + dy*dy                           (parents a, b)
//   K     = (S - d^2)(d^2 - Dm),  S = (ra+rb)^2, Dm = (ra-rb)^2   (16 area^2, Heron)
//   h     = sqrt(K) / (2 d),  f = (d^2 + ra^2 - rb^2) / (2 d)    (height and its foot)
//   base  = p_a + (f/d)(dx, dy),  off = (h/d)(-dy, dx)
//   p     = base + off or base - off, the one nearer the previous position (tie: +)
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

// Length drift of the links outside the solve order (rare: only candidates with
// redundant links).  Returns true when one of them moved by more than thr.
__device__ bool drift_check(const SimArgs& A, int cand, int D, int n, const double2* P, int bd, int tid,
                            double thr) {
  const int J = A.J;
  const uint32_t* adj = A.adj + (size_t)cand * J;
  const uint8_t* sj = A.slot_joint + (size_t)cand * J;
  const DyadF32* df = A.df + (size_t)cand * J;
  const double* x0 = A.x0 + (size_t)cand * J * 2;
  const int pivot = A.motor[2 * cand], tip = A.motor[2 * cand + 1];
  const uint32_t fixed = A.fixed[cand];
  for (int si = 0; si < n; ++si) {
    const int ji = sj[si];
    for (int sk = 0; sk < n; ++sk) {
      const int jk = sj[sk];
      if (jk <= ji || !((adj[ji] >> jk) & 1u)) continue;
      if ((ji == pivot && jk == tip) || (ji == tip && jk == pivot)) continue;
      bool parent_edge = false;
      if (si < D) {
        uint32_t q = df[si].slots;
        parent_edge |= (int)(q & 0xFF) == sk || (int)((q >> 8) & 0xFF) == sk;
      }
      if (sk < D) {
        uint32_t q = df[sk].slots;
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

template <int DMAX, int SRC>
__global__ void __launch_bounds__(256) sim64_kernel(SimArgs A) {
  extern __shared__ unsigned char smem[];
  const int bd = blockDim.x;
  const int tid = threadIdx.x;
  double2* P = reinterpret_cast<double2*>(smem);  // [nslot][bd]
  const int T = A.T;
  const int J = A.J;
  const bool want_path = A.path != nullptr;
  const int cnt_next = SRC == kFromEsc ? kCntEscNext : SRC == kFromRefine ? kCntRefineNext : kCntNext;
  const int cnt_items = SRC == kFromEsc ? kCntEsc : SRC == kFromRefine ? kCntRefine : kCntItems;

  int cand = -1, t = 0, D = 0, n = 0, out_slot = 0;
  bool no_path = true, redundant = false, prefix_bad = false;
  double px = 0, py = 0, vx = 0, vy = 0, deg_thr = 0, drift_thr = 0;
  bool exhausted = false;

  for (;;) {
    uint64_t idle = __ballot(cand < 0);
    int nidle = __popcll(idle);
    if (nidle == kWave && exhausted) break;
    if (!exhausted && nidle > 0) {
      int leader = __ffsll((unsigned long long)idle) - 1;
      int base = 0;
      if (__lane_id() == leader) base = atomicAdd(&A.counters[cnt_next], nidle);
      base = __shfl(base, leader);
      const int items = A.counters[cnt_items];
      if (base + nidle >= items) exhausted = true;
      if (cand < 0) {
        int p = base + mbcnt64(idle);
        if (p < items) {
          int c;
          int t0 = 0;
          bool from_x0 = true;
          prefix_bad = false;
          if (SRC == kFromEsc) {
            EscEntry e = A.esc[p];
            c = e.cand;
            t0 = e.t;
            from_x0 = e.from_x0 != 0;
            prefix_bad = e.path_bad != 0;
          } else if (SRC == kFromRefine) {
            c = A.refine[p];
          } else {
            c = A.perm[p];
          }
          cand = c;
          t = t0;
          CandMeta m = A.meta[c];
          D = m.D;
          n = m.n;
          out_slot = m.out_slot;
          no_path = (m.flags & kFlagNoPath) != 0;
          redundant = (m.flags & kFlagRedundant) != 0;
          CandF64 f = A.cd[c];
          px = f.px;
          py = f.py;
          vx = f.vx;
          vy = f.vy;
          deg_thr = f.deg_thr;
          drift_thr = f.drift_thr;
          const uint8_t* sj = A.slot_joint + (size_t)c * J;
          const double* x0 = A.x0 + (size_t)c * J * 2;
          const float2* dump = SRC == kFromEsc ? A.esc_pos + (size_t)p * J : nullptr;
          for (int sl = 0; sl < n; ++sl) {
            double2 v;
            if (sl > D || from_x0) {  // fixed joints, or reference positions at t = 0
              const int j = sj[sl];
              v = make_double2(x0[2 * j], x0[2 * j + 1]);
            } else {
              const float2 q = dump[sl];
              v = make_double2((double)q.x, (double)q.y);
            }
            P[sl * bd + tid] = v;
          }
        }
      }
    }
    if (cand >= 0) {
      const double2 cs = A.cs64[t];
      const double ct = cs.x, st = cs.y;
      P[D * bd + tid] = make_double2(px + (ct * vx - st * vy), py + (st * vx + ct * vy));
      const DyadF32* df = A.df + (size_t)cand * J;
      const DyadF64* dd = A.dd + (size_t)cand * J;
      int fail = 0;
#pragma unroll
      for (int s = 0; s < DMAX; ++s) {
        if (s < D && fail == 0) {
          const uint32_t sl = df[s].slots;
          const DyadF64 q = dd[s];
          const int a = sl & 0xFF, b = (sl >> 8) & 0xFF;
          const double2 pa = P[a * bd + tid];
          const double2 pb = P[b * bd + tid];
          const double dx = pb.x - pa.x;
          const double dy = pb.y - pa.y;
          const double d2 = dx * dx + dy * dy;
          if (d2 <= deg_thr) {
            fail = 2;
          } else {
            const double K = (q.S - d2) * (d2 - q.Dm);
            if (K < 0.0) {
              fail = 1;
            } else {
              const double d = sqrt(d2);
              const double h = sqrt(K) / (2.0 * d);
              const double along = (d2 + q.ra2 - q.rb2) / (2.0 * d);
              const double bx = pa.x + (along / d) * dx;
              const double by = pa.y + (along / d) * dy;
              const double ox = -(h / d) * dy;
              const double oy = (h / d) * dx;
              const double cpx = bx + ox, cpy = by + oy;
              const double cmx = bx - ox, cmy = by - oy;
              const double2 pr = P[s * bd + tid];
              const double dp2 = (pr.x - cpx) * (pr.x - cpx) + (pr.y - cpy) * (pr.y - cpy);
              const double dm2 = (pr.x - cmx) * (pr.x - cmx) + (pr.y - cmy) * (pr.y - cmy);
              P[s * bd + tid] = dp2 <= dm2 ? make_double2(cpx, cpy) : make_double2(cmx, cmy);
            }
          }
        }
      }
      if (fail == 0 && redundant && drift_check(A, cand, D, n, P, bd, tid, drift_thr)) fail = 3;
      bool done = false;
      if (fail != 0) {
        A.status[cand] = (uint8_t)fail;
        A.fail_step[cand] = (int16_t)t;
        if (SRC == kFromEsc && prefix_bad && A.write_all)
          A.refine[atomicAdd(&A.counters[kCntRefine], 1)] = cand;
        done = true;
      } else {
        if (want_path && !no_path) {
          const double2 po = P[out_slot * bd + tid];
          if (A.path_f64)
            reinterpret_cast<double2*>(A.path)[(size_t)cand * T + t] = po;
          else
            reinterpret_cast<float2*>(A.path)[(size_t)cand * T + t] = make_float2((float)po.x, (float)po.y);
        }
        if (++t == T) {
          A.status[cand] = 0;
          A.fail_step[cand] = -1;
          if (SRC == kFromEsc && prefix_bad) A.refine[atomicAdd(&A.counters[kCntRefine], 1)] = cand;
          done = true;
        }
      }
      if (done) cand = -1;
    }
  }
}

template <int DMAX, int SRC>
void launch_one(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  const int bd = cfg.waves * kWave;
  const size_t lds = (size_t)a.nslot * bd * sizeof(double2);
  hipLaunchKernelGGL((sim64_kernel<DMAX, SRC>), dim3(cfg.grid), dim3(bd), lds, st, a);
}

template <int SRC>
hipError_t dispatch(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  switch (sim32_dmax(a.J)) {
    case 5: launch_one<5, SRC>(a, cfg, st); break;
    case 11: launch_one<11, SRC>(a, cfg, st); break;
    case 18: launch_one<18, SRC>(a, cfg, st); break;
    default: launch_one<30, SRC>(a, cfg, st); break;
  }
  return hipGetLastError();
}

template <int DMAX, int SRC>
int occ(int waves, int lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sim64_kernel<DMAX, SRC>, waves * kWave, lds) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <int SRC>
int occ_for(int J, int waves, int lds) {
  switch (sim32_dmax(J)) {
    case 5: return occ<5, SRC>(waves, lds);
    case 11: return occ<11, SRC>(waves, lds);
    case 18: return occ<18, SRC>(waves, lds);
    default: return occ<30, SRC>(waves, lds);
  }
}

}  // namespace

int sim64_lds_bytes(int nslot, int waves) { return nslot * waves * kWave * (int)sizeof(double2); }

hipError_t launch_sim64(const SimArgs& a, int source, const LaunchCfg& cfg, hipStream_t st) {
  switch (source) {
    case kFromEsc: return dispatch<kFromEsc>(a, cfg, st);
    case kFromRefine: return dispatch<kFromRefine>(a, cfg, st);
    default: return dispatch<kFromPerm>(a, cfg, st);
  }
}

int sim64_blocks_per_cu(int J, int source, int waves, int lds) {
  switch (source) {
    case kFromEsc: return occ_for<kFromEsc>(J, waves, lds);
    case kFromRefine: return occ_for<kFromRefine>(J, waves, lds);
    default: return occ_for<kFromPerm>(J, waves, lds);
  }
}

}  // namespace links
