// simwave.hip -- the FP64 passes with one candidate per wave and its joint
// positions in registers.
//
// The parallel-in-time passes of sim64.hip give one candidate to a segment of
// lanes; each lane keeps its own column of positions in LDS, which limits them to
// one and a half to two waves per SIMD.  Here the whole wave holds one candidate:
// lane r computes step t0 - 1 + r (lane 0, the provider, holds the starting
// positions or recomputes the last decided step), so every slot index the solve
// order names (Methodology, "Graphical Simulator") is the same in all lanes, and
// a lane's positions live in four vectors of 32-bit registers (x and y, low and
// high words) read and written at that uniform index.  The per-entry constants
// are loaded once per candidate, entry s into lane s, and read with readlane.
// The continuity rule compares each lane's placement with its left neighbour's
// (a whole-wave DPP shift); the first lane in step order with a failure, a link
// drift or a side change ends the round exactly as in the segmented passes, so
// statuses, failure steps, side records and rows are the same bit for bit.
#include "common.h"
#include "kernels.h"

namespace links {

namespace {

enum : int { kWvNone = 0, kWvLock = 1, kWvDegenerate = 2, kWvDrift = 3, kWvSide = 4 };

// steps a round decides: lanes 1 .. 63
constexpr int kWvStep = kWave - 1;
// hand-over queue entries a wave claims with one atomic
constexpr int kWvClaim = 4;

// The positions of every slot at this lane's step.  A vector of registers above
// 12 words is allocated as 16 or 32 words, so more than 16 slots are held as a
// 16-slot part and a part for the rest (80 registers for 20 slots rather than
// 128), the part chosen by a branch on the uniform index.
template <int N>
struct RegPart {
  typedef uint32_t V __attribute__((ext_vector_type(N)));
  V xl, xh, yl, yh;
  __device__ __forceinline__ double2 get(int i) const {
    return make_double2(__hiloint2double((int)xh[i], (int)xl[i]), __hiloint2double((int)yh[i], (int)yl[i]));
  }
  __device__ __forceinline__ void put(int i, double2 v) {
    xl[i] = (uint32_t)__double2loint(v.x);
    xh[i] = (uint32_t)__double2hiint(v.x);
    yl[i] = (uint32_t)__double2loint(v.y);
    yh[i] = (uint32_t)__double2hiint(v.y);
  }
};

template <int NS>
struct RegSlots {
  static constexpr int N0 = NS > 16 ? 16 : NS;
  static constexpr int N1 = NS > 16 ? NS - 16 : 1;
  RegPart<N0> lo;
  RegPart<N1> hi;
  __device__ __forceinline__ double2 get(int i) const {
    if (NS <= 16 || i < 16) return lo.get(i);
    return hi.get(i - 16);
  }
  __device__ __forceinline__ void put(int i, double2 v) {
    if (NS <= 16 || i < 16)
      lo.put(i, v);
    else
      hi.put(i - 16, v);
  }
};

// the value held by lane - 1 (lane 0 gets 0)
__device__ __forceinline__ double wave_prev(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// the fast variant's 1/sqrt(x), as in the segmented passes: hardware estimate and
// one Newton step
__device__ __forceinline__ double rsqrt_w(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  return y * fma(-hx * y, y, 1.5);
}

__device__ __forceinline__ double sqd_w(double ax, double ay, double bx, double by) {
  const double dx = ax - bx;
  const double dy = ay - by;
  return dx * dx + dy * dy;
}

// Length drift of the links outside the solve order (candidates with redundant
// links): true when one of them moved by more than thr.  Every index is uniform.
template <int NS>
__device__ bool drift_wave(const SimArgs& A, int cand, int item, int D, int n, const RegSlots<NS>& P, double thr) {
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
      const double L = sqrt(sqd_w(x0[2 * ji], x0[2 * ji + 1], x0[2 * jk], x0[2 * jk + 1]));
      const double2 pi = P.get(si), pk = P.get(sk);
      const double now = sqrt(sqd_w(pi.x, pi.y, pk.x, pk.y));
      if (fabs(now - L) > thr) return true;
    }
  }
  return false;
}

template <int DMAX, int SRC, bool EXACT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
simwave64_kernel(SimArgs A) {
  constexpr int NS = DMAX + 2;  // slots: the placed joints, the tip and the fixed joints
  const int lane = __lane_id();
  const int T = A.T;
  const int J = A.J;
  const int Bs = A.Bs;
  const int cnt_next = SRC == kFromEsc ? kCntEscNext : SRC == kFromPath ? kCntPathNext : kCntNext;
  const int cnt_items = SRC == kFromEsc ? kCntEsc : SRC == kFromPath ? kCntPath : kCntItems;
  const int items = __builtin_amdgcn_readfirstlane(A.counters[cnt_items]);
  const bool orient = A.branch != 0;  // sides fixed at the start (else continuity)
  RegSlots<NS> P;
#pragma unroll
  for (int i = 0; i < NS; ++i) P.put(i, make_double2(0.0, 0.0));

  int cur = 0, left = 0;
  for (;;) {
    if (left == 0) {
      int base = 0;
      if (lane == 0) base = atomicAdd(&A.counters[cnt_next], kWvClaim);
      base = __builtin_amdgcn_readfirstlane(base);
      if (base >= items) break;
      cur = base;
      left = min(kWvClaim, items - base);
    }
    const int p = cur++;
    --left;

    // ---- the candidate of list entry p (every value here is the same in all lanes)
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
    it = __builtin_amdgcn_readfirstlane(it);
    ts = __builtin_amdgcn_readfirstlane(ts);
    const int c = __builtin_amdgcn_readfirstlane(A.perm[it]);
    const CandMeta m = A.meta[it];
    const int D = __builtin_amdgcn_readfirstlane((int)m.D);
    const int n = __builtin_amdgcn_readfirstlane((int)m.n);
    const int out_slot = __builtin_amdgcn_readfirstlane((int)m.out_slot);
    const int flags = __builtin_amdgcn_readfirstlane((int)m.flags);
    int t_end = T;
    int64_t row = -1;
    if (SRC == kFromPath) {
      if (flags & kFlagNoPath) continue;
      row = A.write_all ? (int64_t)c : (int64_t)A.path_row[c];
      const int fs = A.fail_step[c];
      if (fs >= 0) t_end = fs;  // the path exists up to the failing step
      if (row < 0 || t_end <= 0) continue;
    }
    const bool redundant = (flags & kFlagRedundant) != 0;
    const CandF64 f = A.cd[it];
    const double px = f.px, py = f.py, vx = f.vx, vy = f.vy;
    const double deg_thr = f.deg_thr, drift_thr = f.drift_thr;

    // entry s's constants in lane s: S, Dm and ra^2, rb^2 (EXACT) or
    // Kc = (ra^2 - rb^2)/2 (fast), and its parent slots
    double qS = 0.0, qDm = 0.0, qA = 0.0, qB = 0.0;
    uint32_t qsl = 0u;
    if (lane < D) {
      const DyadF64 q = A.dd[(size_t)lane * Bs + it];
      qS = q.S;
      qDm = q.Dm;
      qA = EXACT ? q.ra2 : 0.5 * (q.ra2 - q.rb2);
      qB = q.rb2;
      qsl = A.df[(size_t)lane * Bs + it].slots;
    }
    // starting positions (the reference of the first round): slot k in lane k,
    // then every slot broadcast to all lanes
    double2 v0 = make_double2(0.0, 0.0);
    if (lane < n) {
      if (lane > D || from_x0) {
        const int j = A.slot_joint[(size_t)lane * Bs + it];
        v0 = reinterpret_cast<const double2*>(A.x0 + (size_t)c * J * 2)[j];
      } else {
        const float2 w = A.esc_pos[(size_t)it * J + lane];
        v0 = make_double2((double)w.x, (double)w.y);
      }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (k < n) P.put(k, make_double2(lane_d(v0.x, k), lane_d(v0.y, k)));

    // first guess of the sides: those of the starting positions
    uint32_t og = 0u;
    for (int s = 0; s < D; ++s) {
      const uint32_t sl = (uint32_t)__builtin_amdgcn_readlane((int)qsl, s);
      const double2 pa = P.get(sl & 0xFF), pb = P.get((sl >> 8) & 0xFF), pk = P.get(s);
      if ((pb.x - pa.x) * (pk.y - pa.y) - (pb.y - pa.y) * (pk.x - pa.x) >= 0.0) og |= 1u << s;
    }
    uint32_t ori = orient ? (uint32_t)f.side : og;  // side of every dyad for the computing lanes
    uint32_t ori_prov = ori;                          // the sides in force at the provider's step
    bool fresh = true;                                // the provider holds the starting positions
    int t0 = ts, restarts = 0;

    for (;;) {
      // ---- one round: lane r computes step t0 - 1 + r
      const int t = t0 - 1 + lane;
      const bool comp = t < t_end && !(lane == 0 && fresh);
      const uint32_t side = lane == 0 ? ori_prov : ori;
      {
        // (the slot vectors are written unconditionally, a lane that does not
        // compute keeping its value, so that no copy of them is made per branch)
        const double2 cs = A.cs64[comp ? t : 0];
        const double ct = cs.x, st = cs.y;
        double2 tipv;
        if (EXACT)
          tipv = make_double2(px + (ct * vx - st * vy), py + (st * vx + ct * vy));
        else
          tipv = make_double2(fma(ct, vx, fma(-st, vy, px)), fma(st, vx, fma(ct, vy, py)));
        const double2 old = P.get(D);
        P.put(D, comp ? tipv : old);
      }
      int ev = kWvNone, ev_s = 0;
      for (int s = 0; s < D; ++s) {
        const uint32_t sl = (uint32_t)__builtin_amdgcn_readlane((int)qsl, s);
        const double S = lane_d(qS, s), Dm = lane_d(qDm, s), cA = lane_d(qA, s), cB = lane_d(qB, s);
        const bool act = comp && ev == kWvNone;
        double2 val = P.get(s);
        const double2 pa = P.get(sl & 0xFF);
        const double2 pb = P.get((sl >> 8) & 0xFF);
        // EXACT: both intersections; fast: base point and offset
        double rx0 = 0, ry0 = 0, rx1 = 0, ry1 = 0;
        bool placed = false;
        if (act) {
          const double dx = pb.x - pa.x;
          const double dy = pb.y - pa.y;
          const bool lft = (side >> s) & 1u;
          if (EXACT) {
            const double d2 = dx * dx + dy * dy;
            if (d2 <= deg_thr) {
              ev = kWvDegenerate;
            } else {
              const double K = (S - d2) * (d2 - Dm);
              if (K < 0.0) {
                ev = kWvLock;
              } else {
                const double d = sqrt(d2);
                const double h = sqrt(K) / (2.0 * d);
                const double along = (d2 + cA - cB) / (2.0 * d);
                const double bx = pa.x + (along / d) * dx;
                const double by = pa.y + (along / d) * dy;
                const double ox = -(h / d) * dy;
                const double oy = (h / d) * dx;
                rx0 = bx + ox;
                ry0 = by + oy;
                rx1 = bx - ox;
                ry1 = by - oy;
                val = lft ? make_double2(rx0, ry0) : make_double2(rx1, ry1);
                placed = true;
              }
            }
          } else {
            const double d2 = fma(dy, dy, dx * dx);
            const double K = (S - d2) * (d2 - Dm);
            if (d2 <= deg_thr) {
              ev = kWvDegenerate;
            } else if (K < 0.0) {
              ev = kWvLock;
            } else {
              const double rd = rsqrt_w(d2);
              const double inv = rd * rd;
              const double Kp = fmax(K, 1e-300);
              const double sK = Kp * rsqrt_w(Kp);
              const double al = fma(cA, inv, 0.5);
              const double be = sK * (0.5 * inv);
              rx0 = fma(al, dx, pa.x);
              ry0 = fma(al, dy, pa.y);
              rx1 = -be * dy;
              ry1 = be * dx;
              const double sgn = lft ? 1.0 : -1.0;
              val = make_double2(fma(sgn, rx1, rx0), fma(sgn, ry1, ry0));
              placed = true;
            }
          }
        }
        P.put(s, val);
        // the previous step's position of this joint, from the left neighbour
        const double qx = wave_prev(val.x), qy = wave_prev(val.y);
        if (placed && lane > 0 && !orient) {
          bool rule_left;
          if (EXACT) {
            const double dp2 = (qx - rx0) * (qx - rx0) + (qy - ry0) * (qy - ry0);
            const double dm2 = (qx - rx1) * (qx - rx1) + (qy - ry1) * (qy - ry1);
            rule_left = dp2 <= dm2;
          } else {
            rule_left = fma(qx - rx0, rx1, (qy - ry0) * ry1) >= 0.0;
          }
          if (rule_left != (((side >> s) & 1u) != 0u)) {
            ev = kWvSide;
            ev_s = s;
          }
        }
      }
      if (comp && lane > 0 && ev == kWvNone && redundant && drift_wave(A, c, it, D, n, P, drift_thr))
        ev = kWvDrift;

      // ---- the first event in step order
      const uint64_t evb = __ballot(comp && lane > 0 && ev != kWvNone);
      const int fl = evb ? __ffsll((unsigned long long)evb) - 1 : kWave;
      const int info = fl < kWave ? __builtin_amdgcn_readlane(ev | (ev_s << 8), fl) : 0;
      const int kind = fl < kWave ? (info & 0xFF) : kWvNone;
      // the sides of each decided step that ends a chunk of a path row, for the
      // chunked path pass
      if (SRC != kFromPath && A.side_ck != nullptr && comp && lane > 0 && lane < fl && t + 1 < T &&
          ((t + 1) & (kPathChunk - 1)) == 0)
        A.side_ck[(size_t)c * A.ck_n + (t + 1) / kPathChunk] = side;
      if (SRC == kFromPath && comp && lane > 0 && lane < fl) {
        const double2 po = P.get(out_slot);
        if (A.path_f64)
          reinterpret_cast<double2*>(A.path)[row * T + t] = po;
        else
          reinterpret_cast<float2*>(A.path)[row * T + t] = make_float2((float)po.x, (float)po.y);
      }
      const int te = t0 - 1 + fl;  // step of the event
      if (kind == kWvNone) {
        const int next = t0 + kWvStep;
        if (next >= t_end) {
          if (SRC != kFromPath && lane == 0) {
            A.status[c] = 0;
            A.fail_step[c] = -1;
            if (SRC == kFromPerm && A.esc_step) A.esc_step[c] = -1;
          }
          break;
        }
        t0 = next;
        ori_prov = ori;
        fresh = false;
        restarts = 0;
      } else if (kind == kWvSide) {
        // the provider of the restarted round is the step before the change
        if (fl >= 2) {
          ori_prov = ori;
          fresh = false;
          restarts = 0;
        }
        ori ^= 1u << (info >> 8);
        t0 = te;
        if (++restarts > D + 1) {
          // cannot happen (each restart at one step moves the first change to a
          // later dyad); the candidate is left without a final status
          if (SRC != kFromPath && lane == 0) A.status[c] = kPending;
          break;
        }
      } else {
        if (SRC == kFromPath) {
          // a failure here (possible only within rounding of a threshold) leaves the
          // rest of the row NaN
          const double nan = __builtin_nan("");
          for (int tt = te + lane; tt < t_end; tt += kWave) {
            if (A.path_f64)
              reinterpret_cast<double2*>(A.path)[row * T + tt] = make_double2(nan, nan);
            else
              reinterpret_cast<float2*>(A.path)[row * T + tt] = make_float2((float)nan, (float)nan);
          }
        } else if (lane == 0) {
          A.status[c] = (uint8_t)kind;
          A.fail_step[c] = (int16_t)te;
          if (SRC == kFromPerm && A.esc_step) A.esc_step[c] = -1;
        }
        break;
      }
    }
  }
}

template <int DMAX, int SRC, bool EXACT>
void launch_wave_one(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  hipLaunchKernelGGL((simwave64_kernel<DMAX, SRC, EXACT>), dim3(cfg.grid), dim3(cfg.waves * kWave), 0, st, a);
}

template <int SRC, bool EXACT>
hipError_t dispatch_wave(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  switch (sim32_dmax(a.J)) {
    case 5: launch_wave_one<5, SRC, EXACT>(a, cfg, st); break;
    case 11: launch_wave_one<11, SRC, EXACT>(a, cfg, st); break;
    case 18: launch_wave_one<18, SRC, EXACT>(a, cfg, st); break;
    default: return hipErrorInvalidValue;  // more than 20 joints: the segmented passes
  }
  return hipGetLastError();
}

template <int DMAX, int SRC, bool EXACT>
int occ_wave(int waves) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, simwave64_kernel<DMAX, SRC, EXACT>, waves * kWave, 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <int SRC, bool EXACT>
int occ_wave_for(int J, int waves) {
  switch (sim32_dmax(J)) {
    case 5: return occ_wave<5, SRC, EXACT>(waves);
    case 11: return occ_wave<11, SRC, EXACT>(waves);
    default: return occ_wave<18, SRC, EXACT>(waves);
  }
}

}  // namespace

bool sim64_wave_fits(int J) { return sim32_dmax(J) <= 18; }

hipError_t launch_sim64_wave(const SimArgs& a, int source, bool exact, const LaunchCfg& cfg, hipStream_t st) {
  if (exact) {
    switch (source) {
      case kFromEsc: return dispatch_wave<kFromEsc, true>(a, cfg, st);
      case kFromPath: return dispatch_wave<kFromPath, true>(a, cfg, st);
      default: return dispatch_wave<kFromPerm, true>(a, cfg, st);
    }
  }
  switch (source) {
    case kFromEsc: return dispatch_wave<kFromEsc, false>(a, cfg, st);
    case kFromPath: return dispatch_wave<kFromPath, false>(a, cfg, st);
    default: return dispatch_wave<kFromPerm, false>(a, cfg, st);
  }
}

int sim64_wave_blocks_per_cu(int J, int source, bool exact, int waves) {
  if (exact) {
    switch (source) {
      case kFromEsc: return occ_wave_for<kFromEsc, true>(J, waves);
      case kFromPath: return occ_wave_for<kFromPath, true>(J, waves);
      default: return occ_wave_for<kFromPerm, true>(J, waves);
    }
  }
  switch (source) {
    case kFromEsc: return occ_wave_for<kFromEsc, false>(J, waves);
    case kFromPath: return occ_wave_for<kFromPath, false>(J, waves);
    default: return occ_wave_for<kFromPerm, false>(J, waves);
  }
}

}  // namespace links
