// sim32.hip -- FP32 validity pass: one candidate per lane, persistent waves that
// refill idle lanes from a work list sorted by solve-order length.
//
// Per actuator step t (theta_t = 2 pi t / T; Methodology, "Dataset Features &
// Statistics", item 2) the tip is turned about the pivot and every joint of the
// solve order (Methodology, "Graphical Simulator") is placed at an intersection
// of the circles about its two parents.  The mechanism locks when the circles miss
// (Methodology, "Finding Valid Initial Positions").
//
// Each lane keeps its joints in an LDS column laid out [slot][lane] (conflict-free
// for 8-byte accesses whatever slot each lane reads) together with a first-order
// bound on the FP32 error of every joint.  A placement with parents a, b amplifies
// their error by 1/sin(gamma) = 2 ra rb / sqrt(K), gamma being the angle between
// the two links at the placed joint.  A decision (lock, branch side) is taken in
// FP32 only when its margin exceeds both the stated band and the propagated error
// bound; otherwise the lane stops, dumps its column and hands the candidate to the
// FP64 pass at that step ("escalation").
#include "common.h"
#include "kernels.h"

namespace links {

namespace {

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <int DMAX, int MODE>
__global__ void __launch_bounds__(256) sim32_kernel(SimArgs A) {
  extern __shared__ unsigned char smem[];
  const int bd = blockDim.x;
  const int tid = threadIdx.x;
  float2* P = reinterpret_cast<float2*>(smem);  // [nslot][bd]
  float* E = reinterpret_cast<float*>(P + (size_t)A.nslot * bd);
  const int T = A.T;
  const int J = A.J;
  const bool want_path = A.path != nullptr;

  int cand = -1, t = 0, D = 0, n = 0, out_slot = 0;
  bool no_path = true;
  float px = 0.f, py = 0.f, vx = 0.f, vy = 0.f, U = 0.f, KB = 0.f, CD = 0.f, EB = 0.f, EP = 0.f;
  float U2 = 0.f, TS = 0.f, uu = 0.f, DG = 0.f;
  bool force64 = false, path_bad = false;
  float cS[DMAX], cDm[DMAX], cKc[DMAX];
  uint32_t cSl[DMAX];
#pragma unroll
  for (int s = 0; s < DMAX; ++s) {
    cS[s] = 0.f;
    cDm[s] = 0.f;
    cKc[s] = 0.f;
    cSl[s] = 0u;
  }
  bool exhausted = false;

  for (;;) {
    // ---------------- refill idle lanes (wave-uniform control flow)
    uint64_t idle = __ballot(cand < 0);
    int nidle = __popcll(idle);
    if (nidle == kWave && exhausted) break;
    if (!exhausted && nidle > 0 && (nidle >= A.refill_min || nidle == kWave)) {
      int leader = __ffsll((unsigned long long)idle) - 1;
      int base = 0;
      if (lane_id() == leader) base = atomicAdd(&A.counters[kCntNext], nidle);
      base = __shfl(base, leader);
      const int items = A.counters[kCntItems];
      if (base + nidle >= items) exhausted = true;
      if (cand < 0) {
        int p = base + mbcnt64(idle);
        if (p < items) {
          int c = A.perm[p];
          cand = c;
          t = 0;
          path_bad = false;
          CandMeta m = A.meta[c];
          D = m.D;
          n = m.n;
          out_slot = m.out_slot;
          no_path = (m.flags & kFlagNoPath) != 0;
          force64 = (m.flags & kFlagRedundant) != 0;  // drift checks run in the FP64 pass
          CandF32 f = A.cf[c];
          px = f.px;
          py = f.py;
          vx = f.vx;
          vy = f.vy;
          U = f.U;
          KB = f.KB;
          CD = f.CD;
          EB = f.EB;
          EP = f.EP;
          U2 = f.U2;
          TS = f.TS;
          uu = f.u;
          DG = f.DG;
          const DyadF32* df = A.df + (size_t)c * J;
#pragma unroll
          for (int s = 0; s < DMAX; ++s) {
            if (s < D) {
              DyadF32 q = df[s];
              cS[s] = q.S;
              cDm[s] = q.Dm;
              cKc[s] = q.Kc;
              cSl[s] = q.slots;
            }
          }
          const float2* xs = A.x0s + (size_t)c * J;
          for (int sl = 0; sl < n; ++sl) {
            const float2 q = xs[sl];
            P[sl * bd + tid] = q;
            E[sl * bd + tid] = uu * (fabsf(q.x) + fabsf(q.y));  // rounding of x0 to FP32
          }
        }
      }
      if (__ballot(cand >= 0) == 0ull) {
        if (exhausted) break;
        continue;
      }
    }
    if (cand < 0) continue;
    {
    // ---------------- one actuator step of this lane's candidate
    const float2 cs = A.cs32[t];
    const float tx = fmaf(cs.x, vx, fmaf(-cs.y, vy, px));
    const float ty = fmaf(cs.y, vx, fmaf(cs.x, vy, py));
    P[D * bd + tid] = make_float2(tx, ty);
    E[D * bd + tid] = U;

    bool ev = force64, lock_ev = false;
    int lock_kind = 1;
#pragma unroll
    for (int s = 0; s < DMAX; ++s) {
      if (s < D && !ev) {
        const uint32_t sl = cSl[s];
        const int a = sl & 0xFF, b = (sl >> 8) & 0xFF;
        const float2 pa = P[a * bd + tid];
        const float2 pb = P[b * bd + tid];
        const float2 pr = P[s * bd + tid];
        const float Ea = E[a * bd + tid];
        const float Eb = E[b * bd + tid];
        const float Ep = E[s * bd + tid];
        const float dx = pb.x - pa.x, dy = pb.y - pa.y;
        const float d2 = fmaf(dy, dy, dx * dx);
        const float S = cS[s], Dm = cDm[s];
        // discriminant of the circle-circle intersection, 16 area^2 (Heron)
        const float K = (S - d2) * (d2 - Dm);
        const float rd = rsq(d2);      // 1/d
        const float inv = rd * rd;     // 1/d^2
        const float Kp = fmaxf(K, 1e-30f);
        const float rK = rsq(Kp);
        const float sK = Kp * rK;      // sqrt(K)
        const float be = sK * (0.5f * inv);           // h/d
        const float al = fmaf(cKc[s], inv, 0.5f);     // foot of the height along a->b
        const float bx = fmaf(al, dx, pa.x), by = fmaf(al, dy, pa.y);
        const float ox = -be * dy, oy = be * dx;      // left normal, length h
        // branch: the intersection nearer the previous position
        const float sg = fmaf(pr.x - bx, ox, (pr.y - by) * oy);
        const float sgn = sg >= 0.f ? 1.f : -1.f;
        const float nx = fmaf(sgn, ox, bx), ny = fmaf(sgn, oy, by);
        if (MODE == 0) {
          // error bound of the parents and of this placement
          const float Eab = Ea + Eb;
          const float d = d2 * rd;
          const float h = 0.5f * sK * rd;
          const float sensK = 4.f * d * fabsf(fmaf(0.5f, S + Dm, -d2));
          const float kthr = fmaf(sensK, Eab, KB);
          const float mthr = fmaf(Eab, fmaf(TS, rd, 1.f), EB + Ep);
          const bool band = (fabsf(K) < kthr) || (d2 < CD) || (fabsf(sg) < mthr * h);
          if (band) {
            ev = true;
          } else if (K < 0.f) {
            ev = true;
            lock_ev = true;
          } else {
            const float A2 = 0.5f * (S - Dm) * rK;  // 2 ra rb / sqrt(K)
            const float Ek = A2 * (Eab + fmaf(uu, fabsf(pa.x) + fabsf(pa.y), U2));
            P[s * bd + tid] = make_float2(nx, ny);
            E[s * bd + tid] = Ek;
          }
        } else {
          if (d2 <= DG) {
            ev = true;
            lock_ev = true;
            lock_kind = 2;
          } else if (K < 0.f) {
            ev = true;
            lock_ev = true;
          } else {
            P[s * bd + tid] = make_float2(nx, ny);
          }
        }
      }
    }

    bool done = false;
    if (!ev && want_path && !no_path) {
      const float2 po = P[out_slot * bd + tid];
      // the output joint's error bound exceeds the path tolerance: the path of this
      // candidate will be recomputed in FP64 if it is output
      if (MODE == 0 && E[out_slot * bd + tid] > EP) path_bad = true;
      if (A.path_f64) {
        reinterpret_cast<double2*>(A.path)[(size_t)cand * T + t] = make_double2(po.x, po.y);
      } else {
        reinterpret_cast<float2*>(A.path)[(size_t)cand * T + t] = po;
      }
    }
    if (ev) {
      if (lock_ev) {
        A.status[cand] = (uint8_t)lock_kind;
        A.fail_step[cand] = (int16_t)t;
        if (A.esc_step) A.esc_step[cand] = -1;
        if (path_bad && A.write_all) A.refine[atomicAdd(&A.counters[kCntRefine], 1)] = cand;
      } else {
        int i = atomicAdd(&A.counters[kCntEsc], 1);
        EscEntry e;
        e.cand = cand;
        e.t = (int16_t)t;
        e.from_x0 = force64 ? 1 : 0;
        e.path_bad = path_bad ? 1 : 0;
        A.esc[i] = e;
        float2* dump = A.esc_pos + (size_t)i * J;
        for (int sl = 0; sl < n; ++sl) dump[sl] = P[sl * bd + tid];
        if (A.esc_step) A.esc_step[cand] = (int16_t)t;
      }
      done = true;
    } else if (++t == T) {
      A.status[cand] = 0;
      A.fail_step[cand] = -1;
      if (A.esc_step) A.esc_step[cand] = -1;
      if (path_bad) A.refine[atomicAdd(&A.counters[kCntRefine], 1)] = cand;
      done = true;
    }
    if (done) cand = -1;
    }
  }
}

template <int DMAX, int MODE>
void launch_one(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  const int bd = cfg.waves * kWave;
  const size_t lds = (size_t)a.nslot * bd * (sizeof(float2) + sizeof(float));
  hipLaunchKernelGGL((sim32_kernel<DMAX, MODE>), dim3(cfg.grid), dim3(bd), lds, st, a);
}

template <int MODE>
hipError_t dispatch(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  switch (sim32_dmax(a.J)) {
    case 5: launch_one<5, MODE>(a, cfg, st); break;
    case 11: launch_one<11, MODE>(a, cfg, st); break;
    case 18: launch_one<18, MODE>(a, cfg, st); break;
    default: launch_one<30, MODE>(a, cfg, st); break;
  }
  return hipGetLastError();
}

template <int DMAX, int MODE>
int occ(int waves, int lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sim32_kernel<DMAX, MODE>, waves * kWave, lds) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace

int sim32_dmax(int J) {
  // solve-order length is at most J - 2 (the pivot and the tip are not placed)
  if (J <= 7) return 5;
  if (J <= 13) return 11;
  if (J <= 20) return 18;
  return 30;
}

int sim32_lds_bytes(int nslot, int waves) { return nslot * waves * kWave * (int)(sizeof(float2) + sizeof(float)); }

hipError_t launch_sim32(const SimArgs& a, int mode, const LaunchCfg& cfg, hipStream_t st) {
  return mode == 0 ? dispatch<0>(a, cfg, st) : dispatch<1>(a, cfg, st);
}

int sim32_blocks_per_cu(int J, int mode, int waves, int lds) {
  int d = sim32_dmax(J);
  if (mode == 0) {
    switch (d) {
      case 5: return occ<5, 0>(waves, lds);
      case 11: return occ<11, 0>(waves, lds);
      case 18: return occ<18, 0>(waves, lds);
      default: return occ<30, 0>(waves, lds);
    }
  }
  switch (d) {
    case 5: return occ<5, 1>(waves, lds);
    case 11: return occ<11, 1>(waves, lds);
    case 18: return occ<18, 1>(waves, lds);
    default: return occ<30, 1>(waves, lds);
  }
}

}  // namespace links
