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

// a non-negative FP32 bound rounded up to 16 bits (upper half of its encoding)
__device__ __forceinline__ uint16_t bound_up(float e) {
  return (uint16_t)((__float_as_uint(e) + 0xFFFFu) >> 16);
}
__device__ __forceinline__ float bound_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ int mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <int DMAX, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DMAX <= 18 ? 3 : 1)))
sim32_kernel(SimArgs A) {
  extern __shared__ unsigned char smem[];
  const int bd = blockDim.x;
  const int tid = threadIdx.x;
  float2* P = reinterpret_cast<float2*>(smem);  // [nslot][bd]
  // error bounds, stored as the upper 16 bits of the FP32 value rounded up (a
  // bound that is at most 0.4% larger, so it stays a bound)
  uint16_t* E = reinterpret_cast<uint16_t*>(P + (size_t)A.nslot * bd);
  const int T = A.T;
  const int J = A.J;
  // crank table (cos, sin) of every step: in LDS when it fits, so that the step
  // loop issues no global memory operation
  constexpr bool tab_lds = (MODE & 2) == 0;
  float2* tab = reinterpret_cast<float2*>(E + (size_t)A.nslot * bd);
  if (tab_lds) {
    for (int i = tid; i < T; i += bd) tab[i] = A.cs32[i];
    __syncthreads();
  }

  const int Bs = A.Bs;
  int cand = -1, item = 0, t = 0, D = 0, n = 0;
  float px = 0.f, py = 0.f, vx = 0.f, vy = 0.f, U = 0.f, KB = 0.f, CD = 0.f, EB = 0.f;
  float U2 = 0.f, TS = 0.f, DG = 0.f;
  constexpr float uu = kRoundUnit;  // the same for every candidate
  bool force64 = false;
  // A finished candidate's results are written later, for all finished lanes of
  // the wave together (at the next refill or when the wave leaves): its lane is
  // idle meanwhile and keeps its slots in LDS for the hand-over dump.
  // 0 nothing pending, 1 locked, 2 handed over, 3 valid, 4 degenerate; the step of
  // a failure or hand-over stays in t until the results are written
  int fin = 0;
  int fcand = 0;
  constexpr bool orient = (MODE & 8) != 0;  // sides fixed at the start (else continuity)
  uint32_t obits = 0u;                // starting side of each placed joint
  int dmax_w = 0;  // largest solve order among the wave's lanes (uniform)
  float cS[DMAX], cDm[DMAX], cKc[DMAX];
  uint32_t cSl[(DMAX + 1) / 2];  // parent slots, two entries per register
#pragma unroll
  for (int s = 0; s < DMAX; ++s) {
    cS[s] = 0.f;
    cDm[s] = 0.f;
    cKc[s] = 0.f;
  }
#pragma unroll
  for (int s = 0; s < (DMAX + 1) / 2; ++s) cSl[s] = 0u;
  bool exhausted = false;
  // Bucket-affine scheduling: the work list is sorted by solve-order length D
  // (largest first) and split into one bucket per D.  Each wave starts in the
  // bucket that holds its share of the list and refills only from that bucket, so
  // the lanes of a wave place the same number of joints per step; an exhausted
  // bucket sends the wave on to the next smaller bucket that still has work.
  const int* cnt = A.counters;
  const int nwaves = gridDim.x * (blockDim.x / kWave);
  int bucket = 0;
  uint32_t done_mask = 0u;  // buckets this wave has seen exhausted (wave-uniform)
  {
    const int nw = nwaves;
    const int gw = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    const long long items = cnt[kCntItems];
    const long long target = A.spread ? (2LL * gw + 1) * items / (2LL * nw) : 0LL;
    for (int d = kMaxJ - 1; d >= 0; d--) {
      if (cnt[kCntHist + d] == 0) done_mask |= 1u << d;
      else if (cnt[kCntOff + d] <= target) bucket = d;
    }
  }
  // Work is claimed in chunks of A.chunk items held by the wave (one atomic per
  // chunk, not per refill), and the next chunk is claimed ahead: the atomic is
  // issued after a refill's record loads and read only when the wave's current
  // range runs out, so its latency hides behind the steps in between.
  int pre_raw = 0;        // the pending claim's return value (meaningful in lane 0)
  bool pre_pending = false;
  int pre_bucket = 0, pre_req = 0;
  int pre_base = 0, pre_left = 0;    // current range: claimed items not yet handed to lanes
  int next_base = 0, next_left = 0;  // the range after it (from a resolved claim)
  const int rm = A.refill_min;
  const int chunk = A.chunk;

  // next bucket that may still have work: smaller ones first, then larger ones
  auto pick_bucket = [&]() -> bool {
    if (!((done_mask >> bucket) & 1u)) return true;
    for (int d = bucket - 1; d >= 0; --d) {
      if ((done_mask >> d) & 1u) continue;
      const int cur = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(&A.counters[kCntCur + d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (cur < cnt[kCntOff + d] + cnt[kCntHist + d]) {
        bucket = d;
        return true;
      }
      done_mask |= 1u << d;
    }
    for (int d = kMaxJ - 1; d > bucket; --d) {
      if ((done_mask >> d) & 1u) continue;
      const int cur = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(&A.counters[kCntCur + d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (cur < cnt[kCntOff + d] + cnt[kCntHist + d]) {
        bucket = d;
        return true;
      }
      done_mask |= 1u << d;
    }
    return false;
  };

  // results of the finished lanes: one store per result, one atomic for the
  // wave's hand-overs (each lane's queue entry at base + its rank), and the
  // positions of the handed-over candidates at their sorted-position rows
  auto flush = [&]() {
    if (__ballot(fin != 0) == 0ull) return;
    if (fin == 1 || fin == 3 || fin == 4) {
      A.status[fcand] = (uint8_t)(fin == 3 ? 0 : fin == 4 ? 2 : 1);
      A.fail_step[fcand] = (int16_t)(fin == 3 ? -1 : t);
      if (A.esc_step && A.resume != 1) A.esc_step[fcand] = -1;
    }
    const uint64_t em = __ballot(fin == 2);
    if (em != 0ull) {
      const int leader = __ffsll((unsigned long long)em) - 1;
      int base = 0;
      if (lane_id() == leader) base = atomicAdd(A.esc_cnt, __popcll(em));
      base = __shfl(base, leader);
      if (fin == 2) {
        EscEntry e;
        e.item = item;
        e.t = (int16_t)t;
        e.from_x0 = force64 ? 1 : 0;
        e.pad = 0;
        A.esc[base + mbcnt64(em)] = e;
        float2* dump = A.esc_pos + (size_t)item * J;  // the candidate's own row
        for (int sl = 0; sl < n; ++sl) dump[sl] = P[sl * bd + tid];
        if (A.esc_step && A.resume != 1) A.esc_step[fcand] = (int16_t)t;  // the first hand-over
      }
    }
    fin = 0;
  };

  // Drain hand-off: once the work list is exhausted, a wave with fewer than
  // mig_min active lanes stops, and each active lane leaves its column (positions
  // into esc_pos, error bounds into mig_err, at its candidate's sorted position)
  // and (sorted position, next step) in mig_out, counted in *mig_cnt, for the
  // parallel-in-time pass to finish with full segments.
  bool handing = false;  // wave-uniform
  auto hand_off = [&]() {
    const bool live = cand >= 0;
    if (live) {
      float2* dp = A.esc_pos + (size_t)item * J;
      uint16_t* de = A.mig_err + (size_t)item * J;
      for (int sl = 0; sl < n; ++sl) {
        dp[sl] = P[sl * bd + tid];
        de[sl] = E[sl * bd + tid];
      }
    }
    const uint64_t m = __ballot(live);
    if (m != 0ull) {
      const int leader = __ffsll((unsigned long long)m) - 1;
      int base = 0;
      if (lane_id() == leader) base = atomicAdd(A.mig_cnt, __popcll(m));
      base = __shfl(base, leader);
      if (live) {
        EscEntry e;
        e.item = item;
        e.t = (int16_t)t;
        e.from_x0 = 0;
        e.pad = 0;
        A.mig_out[base + mbcnt64(m)] = e;
      }
    }
    cand = -1;
  };

  for (;;) {
    // ---------------- refill idle lanes (wave-uniform control flow)
    uint64_t idle = __ballot(cand < 0);
    int nidle = __popcll(idle);
    if (nidle == kWave && exhausted) {
      flush();
      break;
    }
    if (exhausted && kWave - nidle < A.mig_min) {
      flush();
      handing = true;
      break;
    }
    if (!exhausted && nidle > 0 && (nidle >= rm || nidle == kWave)) {
      flush();  // before new candidates take the finished lanes' slots
      int p = -1;
      // hand out the wave's claimed ranges: the current one, then the next one
      // (resolving the claim made ahead when the current range cannot cover)
      for (int k = 0; k < 2 && nidle > 0; ++k) {
        if (pre_left == 0 && next_left == 0 && pre_pending) {
          const int base = __shfl(pre_raw, 0);
          const int end = cnt[kCntOff + pre_bucket] + cnt[kCntHist + pre_bucket];
          const int got = min(max(end - base, 0), pre_req);
          if (got < pre_req) done_mask |= 1u << pre_bucket;
          next_base = base;
          next_left = got;
          pre_pending = false;
        }
        if (pre_left == 0) {
          pre_base = next_base;
          pre_left = next_left;
          next_left = 0;
        }
        if (pre_left > 0) {
          const int m = min(nidle, pre_left);
          if (cand < 0 && p < 0) {
            const int r = mbcnt64(idle);
            if (r < m) p = pre_base + r;
          }
          pre_base += m;
          pre_left -= m;
          idle = __ballot(cand < 0 && p < 0);
          nidle = __popcll(idle);
        }
      }
      // the rest now; every failed claim marks its bucket done, so this ends
      // within 33 attempts
      for (int attempt = 0; attempt <= kMaxJ && nidle > 0; ++attempt) {
        if (!pick_bucket()) {
          exhausted = true;
          break;
        }
        const int end = cnt[kCntOff + bucket] + cnt[kCntHist + bucket];
        const int leader = __ffsll((unsigned long long)idle) - 1;
        int base = 0;
        if (lane_id() == leader) base = atomicAdd(&A.counters[kCntCur + bucket], nidle);
        base = __shfl(base, leader);
        const int got = min(max(end - base, 0), nidle);
        if (cand < 0 && p < 0) {
          const int r = mbcnt64(idle);
          if (r < got) p = base + r;
        }
        if (got == nidle) break;
        done_mask |= 1u << bucket;  // claimed past its end: exhausted
        idle = __ballot(cand < 0 && p < 0);
        nidle = __popcll(idle);
      }
      if (cand < 0 && p >= 0) {
        {
          // a resume round's work item is an entry of the queue of candidates the
          // FP64 pass returned: its sorted position, next step and positions
          int t0 = 0;
          const float2* init = A.x0s + p;
          size_t init_stride = (size_t)Bs;
          if (A.resume == 1) {
            const EscEntry e = A.res[p];
            init = A.res_pos + (size_t)p * J;
            init_stride = 1;
            t0 = e.t;
            p = e.item;
          }
          const int c = A.perm[p];
          cand = c;
          item = p;
          t = t0;
          CandMeta m = A.meta[p];
          D = m.D;
          n = m.n;
          force64 = (m.flags & kFlagRedundant) != 0;  // drift checks run in the FP64 pass
          CandF32 f = A.cf[p];
          px = f.px;
          py = f.py;
          vx = f.vx;
          vy = f.vy;
          U = f.U;
          KB = f.KB;
          CD = f.CD;
          EB = f.EB;
          U2 = f.U2;
          TS = f.TS;
          DG = f.DG;
          obits = f.side;
#pragma unroll
          for (int s = 0; s < DMAX; ++s) {
            if (s < D) {
              DyadF32 q = A.df[(size_t)s * Bs + p];
              cS[s] = q.S;
              cDm[s] = q.Dm;
              cKc[s] = q.Kc;
              if (s & 1)
                cSl[s >> 1] = (cSl[s >> 1] & 0xFFFFu) | (q.slots << 16);
              else
                cSl[s >> 1] = q.slots & 0xFFFFu;
            }
          }
          // initial positions, a group of slots at a time with the group's loads
          // issued together
          constexpr int NMAX = DMAX + 2;  // joints per candidate at most (J of this template)
          constexpr int G = 4;
#pragma unroll
          for (int g = 0; g < NMAX; g += G) {
            float2 xq[G];
#pragma unroll
            for (int k = 0; k < G; ++k)
              if (g + k < n) xq[k] = init[(size_t)(g + k) * init_stride];
#pragma unroll
            for (int k = 0; k < G; ++k)
              if (g + k < n) {
                P[(g + k) * bd + tid] = xq[k];
                E[(g + k) * bd + tid] = bound_up(uu * (fabsf(xq[k].x) + fabsf(xq[k].y)));  // rounding of x0 to FP32
              }
          }

        }
      }
      // claim the next chunk ahead of time, after the record loads so that
      // nothing waits on it before the current range runs out
      if (!exhausted && !pre_pending && next_left == 0 && pre_left < chunk && !((done_mask >> bucket) & 1u)) {
        // guided size: a share of what remains in the bucket after the current
        // range, split over the waves that work on it, between rm and chunk
        const int end = cnt[kCntOff + bucket] + cnt[kCntHist + bucket];
        const long long wb = max(1LL, (long long)nwaves * cnt[kCntHist + bucket] / max(cnt[kCntItems], 1));
        const int share = (int)((long long)max(end - (pre_base + pre_left), 0) / wb);
        pre_req = min(chunk, max(share, max(rm, 1)));
        pre_bucket = bucket;
        if (lane_id() == 0) pre_raw = atomicAdd(&A.counters[kCntCur + bucket], pre_req);
        pre_pending = true;
      }
      if (__ballot(cand >= 0) == 0ull) {
        if (exhausted) break;
        continue;
      }
      {
        int dm = cand >= 0 ? D : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) dm = max(dm, __shfl_xor(dm, o));
        dmax_w = __builtin_amdgcn_readfirstlane(dm);
      }
    }
    if (cand < 0) continue;
    {
    // ---------------- one actuator step of this lane's candidate
    const float2 cs = tab_lds ? tab[t] : A.cs32[t];
    const float tx = fmaf(cs.x, vx, fmaf(-cs.y, vy, px));
    const float ty = fmaf(cs.y, vx, fmaf(cs.x, vy, py));
    P[D * bd + tid] = make_float2(tx, ty);
    E[D * bd + tid] = bound_up(U);

    bool ev = force64, lock_ev = false;
    int lock_kind = 1;
    uint32_t sb = 0u;  // MODE & 4: the side taken by every placed joint at this step
    // branch-free placement loop: the trip count is the wave's largest solve order
    // (uniform); lanes past their own D or past an event keep their old values
#pragma unroll
    for (int s = 0; s < DMAX; ++s) {
      if (s < dmax_w) {
      const bool act = s < D && !ev;
      const uint32_t sl = (s & 1) ? (cSl[s >> 1] >> 16) : cSl[s >> 1];
      const int a = sl & 0xFF, b = (sl >> 8) & 0xFF;
      const float2 pa = P[a * bd + tid];
      const float2 pb = P[b * bd + tid];
      const float2 pr = P[s * bd + tid];
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
      // continuity: the side of the previous position; orientation: the starting side
      const bool left = orient ? ((obits >> s) & 1u) != 0u : sg >= 0.f;
      if (MODE & 4) sb |= (left ? 1u : 0u) << s;
      const float sgn = left ? 1.f : -1.f;
      const float nx = fmaf(sgn, ox, bx), ny = fmaf(sgn, oy, by);
      bool write;
      float Ek = 0.f, Ep = 0.f;
      if ((MODE & 1) == 0) {
        // error bound of the parents and of this placement
        const float Ea = bound_f(E[a * bd + tid]);
        const float Eb = bound_f(E[b * bd + tid]);
        Ep = bound_f(E[s * bd + tid]);
        const float Eab = Ea + Eb;
        const float d = d2 * rd;
        const float h = 0.5f * sK * rd;
        const float sensK = 4.f * d * fabsf(fmaf(0.5f, S + Dm, -d2));
        // K's own FP32 evaluation (S and Dm rounded from FP64, d^2, the two
        // differences and the product) is within 9 units of (S + d^2)(d^2 + Dm)
        const float kthr = fmaf(sensK, Eab, fmaf(2.5f * uu, (S + d2) * (d2 + Dm), KB));
        // rounding of this placement (foot and normal), as a position error
        const float R = fmaf(uu, fabsf(pa.x) + fabsf(pa.y), U2);
        const float mthr = fmaf(Eab, fmaf(TS, rd, 1.f), EB + Ep + R);
        const bool band = (int)(fabsf(K) < kthr) | (int)(d2 < CD) | (int)(!orient && fabsf(sg) < mthr * h);
        const bool lock = K < 0.f;
        lock_ev = lock_ev | (act & !band & lock);
        ev = ev | (act & (band | lock));
        write = act & !band & !lock;
        const float A2 = 0.5f * (S - Dm) * rK;  // 2 ra rb / sqrt(K)
        Ek = A2 * (Eab + R);
      } else {
        const bool deg = d2 <= DG;
        const bool lock = K < 0.f;
        lock_kind = (act & deg) ? 2 : lock_kind;
        lock_ev = lock_ev | (act & (deg | lock));
        ev = ev | (act & (deg | lock));
        write = act & !deg & !lock;
      }
      P[s * bd + tid] = write ? make_float2(nx, ny) : pr;
      if ((MODE & 1) == 0) E[s * bd + tid] = bound_up(write ? Ek : Ep);
      }
    }

    bool done = false;
    if (ev) {
      fin = lock_ev ? (lock_kind == 2 ? 4 : 1) : 2;
      done = true;
    } else if (++t == T) {
      fin = 3;
      done = true;
    } else if ((MODE & 4) && (t & (kPathChunk - 1)) == 0) {
      // the sides of the step that ends a chunk of the path row (read by the
      // chunked path pass)
      A.side_ck[(size_t)cand * A.ck_n + t / kPathChunk] = sb;
    }
    if (done) {
      fcand = cand;
      cand = -1;
    }
    }
  }
  if (handing) hand_off();
}

template <int DMAX, int MODE>
void launch_one(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  const int bd = cfg.waves * kWave;
  const size_t lds = (size_t)sim32_lds_bytes(a.nslot, cfg.waves, a.T);
  hipLaunchKernelGGL((sim32_kernel<DMAX, MODE>), dim3(cfg.grid), dim3(bd), lds, st, a);
}

template <int MODE>
hipError_t dispatch(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  if (a.T > kTableLds && (MODE & 2) == 0) return dispatch<MODE | 2>(a, cfg, st);
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

// ---- the FP32 pass, parallel in time.
//
// A segment of 16 lanes (one DPP row) holds one candidate; lane r computes step
// t0 - 1 + r, lane 0 (the provider) recomputing the last decided step or holding
// the reference positions, so that each lane finds the previous step's positions
// and error bounds of its candidate in its left neighbour.  Every dyad is placed
// on an assumed side of its parents' line and each computing lane takes the
// decisions of the step-by-step pass (band, lock, branch side) against its
// neighbour's values.  The first lane in step order with a band, a lock or a
// side different from the assumed one ends the pass for the segment: a band hands
// the candidate to FP64 at that step (with the previous step's positions), a lock
// is its outcome, a side change flips the dyad's side and restarts the segment at
// that step.  Lanes before it computed what the step-by-step pass computes.
constexpr int kSeg32 = 16;

__device__ __forceinline__ int row_prev_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false); }
__device__ __forceinline__ float row_prev_f(float v) { return __int_as_float(row_prev_i(__float_as_int(v))); }

enum : int { kE32None = 0, kE32Lock = 1, kE32Degenerate = 2, kE32Band = 3, kE32Side = 4 };

// LDS: positions [nslot][bd] f32x2 and error bounds [nslot][bd] u16; per segment
// two tables of DMAX entries (S, Dm, Kc, parent slots: the live candidate's and the
// next one's), the next candidate's reference positions [32], CandF32 [16],
// meta, index, sorted position and first step, and the reference error bounds
// [32] of a candidate handed on by the step-by-step pass; the crank table when it
// fits.
template <int DMAX>
__host__ __device__ constexpr size_t par32_seg_bytes() {
  return 2 * DMAX * sizeof(float4) + 32 * sizeof(float2) + 16 * sizeof(float) + 4 * sizeof(int) +
         32 * sizeof(uint16_t);
}

template <int DMAX>
__host__ __device__ constexpr size_t par32_lds_bytes(int nslot, int bd, int T) {
  return (size_t)nslot * bd * (sizeof(float2) + sizeof(uint16_t)) + (size_t)(bd / kSeg32) * par32_seg_bytes<DMAX>() +
         (T <= kTableLds ? (size_t)T * sizeof(float2) : 0);
}

template <int DMAX, int MODE>
__global__ void __launch_bounds__(256) simpar32_kernel(SimArgs A) {
  extern __shared__ unsigned char smem[];
  const int bd = blockDim.x;
  const int tid = threadIdx.x;
  float2* P = reinterpret_cast<float2*>(smem);                            // [nslot][bd]
  uint16_t* E = reinterpret_cast<uint16_t*>(P + (size_t)A.nslot * bd);    // [nslot][bd]
  unsigned char* segs = reinterpret_cast<unsigned char*>(E + (size_t)A.nslot * bd);
  unsigned char* seg = segs + (size_t)(tid / kSeg32) * par32_seg_bytes<DMAX>();
  float4* Ct = reinterpret_cast<float4*>(seg);                      // [2][DMAX]
  float2* PN = reinterpret_cast<float2*>(seg + 2 * DMAX * sizeof(float4));  // [32]
  float* CFN = reinterpret_cast<float*>(PN + 32);                   // [16]
  int* MCN = reinterpret_cast<int*>(CFN + 16);                      // meta, index, sorted position, step
  uint16_t* EN = reinterpret_cast<uint16_t*>(MCN + 4);              // [32] bounds of a handed-on candidate
  constexpr bool tab_lds = (MODE & 2) == 0;
  float2* tab = reinterpret_cast<float2*>(segs + (size_t)(bd / kSeg32) * par32_seg_bytes<DMAX>());
  const int T = A.T;
  const int J = A.J;
  const int Bs = A.Bs;
  if (tab_lds) {
    for (int i = tid; i < T; i += bd) tab[i] = A.cs32[i];
    __syncthreads();
  }
  const int lane = __lane_id();
  const int r = lane & (kSeg32 - 1);
  const int seg0 = lane & ~(kSeg32 - 1);

  // segment state (the same in every lane of a segment)
  int cand = -1, item = 0, t0 = 0, D = 0, n = 0, restarts = 0;
  bool fresh = false, force64 = false;
  int cpar = 0;                   // which entry table holds the live candidate
  uint32_t ori = 0u, ori_prov = 0u;
  float px = 0.f, py = 0.f, vx = 0.f, vy = 0.f, U = 0.f, KB = 0.f, CD = 0.f, EB = 0.f;
  float U2 = 0.f, TS = 0.f, uu = 0.f, DG = 0.f;
  int dmax_w = 0;
  const bool orient = A.branch != 0;  // sides fixed at the start (else continuity)
  uint32_t obits = 0u;
  // next candidate: claimed (need_next false), loaded into registers during a
  // pass (in_flight), then staged in LDS (has_staged) until the segment is free
  bool need_next = true, in_flight = false, has_staged = false;
  int pf_p = 0, pf_c = 0;
  uint32_t pf_meta = 0u;
  float pf_cf = 0.f;
  DyadF32 pf_q0, pf_q1;
  float2 pf_w0 = make_float2(0.f, 0.f), pf_w1 = make_float2(0.f, 0.f);
  uint16_t pf_e0 = 0, pf_e1 = 0;
  int pf_t0 = 0;
  pf_q0.S = pf_q0.Dm = pf_q0.Kc = 0.f;
  pf_q0.slots = 0u;
  pf_q1 = pf_q0;
  // hand-over queue entry whose index (an atomic's result) is read one pass later
  bool esc_pend = false;
  int esc_i = 0, esc_item = 0, esc_te = 0;

  const int chunk = A.chunk;
  int cur_base = 0, cur_left = 0;
  bool no_more = false, exhausted = false;
  const int nwaves = gridDim.x * (bd / kWave);
  const int items = A.counters[kCntItems];
  for (;;) {
    // ---- 1. free segments take up their staged candidate (LDS only)
    asm volatile("" ::: "memory");
    const bool fill = cand < 0 && has_staged;
    if (__ballot(fill) != 0ull) {
      if (fill) {
        const uint32_t mp = (uint32_t)MCN[0];
        cand = MCN[1];
        item = MCN[2];
        D = mp & 0xFF;
        n = (mp >> 8) & 0xFF;
        force64 = ((mp >> 24) & kFlagRedundant) != 0;  // drift checks run in the FP64 pass
        px = CFN[0];
        py = CFN[1];
        vx = CFN[2];
        vy = CFN[3];
        U = CFN[4];
        KB = CFN[5];
        CD = CFN[6];
        EB = CFN[7];
        U2 = CFN[8];
        TS = CFN[9];
        uu = CFN[10];
        DG = CFN[11];
        obits = __float_as_uint(CFN[12]);  // CandF32::side
        cpar ^= 1;
        t0 = MCN[3];  // 0, or the next step of a candidate handed on mid-rotation
        fresh = true;
        restarts = 0;
        has_staged = false;
        need_next = true;
#pragma unroll
        for (int sl = 0; sl < DMAX + 2; ++sl)
          if (sl < n) {
            const float2 v = PN[sl];
            P[sl * bd + tid] = v;
            // rounding of x0 to FP32, or the bound a handed-on candidate carried
            E[sl * bd + tid] = A.resume == 2 ? EN[sl] : bound_up(uu * (fabsf(v.x) + fabsf(v.y)));
          }
      }
      __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): LDS operations of a wave complete in order
      asm volatile("" ::: "memory");
      // first guess of the sides: those of the reference positions
      const float4* C = Ct + cpar * DMAX;
      bool g0 = false, g1 = false;
      if (fill) {
        if (r < D) {
          const uint32_t sl = __float_as_uint(C[r].w);
          const float2 pa = P[(sl & 0xFF) * bd + tid], pb = P[((sl >> 8) & 0xFF) * bd + tid], pk = P[r * bd + tid];
          g0 = (pb.x - pa.x) * (pk.y - pa.y) - (pb.y - pa.y) * (pk.x - pa.x) >= 0.f;
        }
        if (r + kSeg32 < D) {
          const uint32_t sl = __float_as_uint(C[r + kSeg32].w);
          const float2 pa = P[(sl & 0xFF) * bd + tid], pb = P[((sl >> 8) & 0xFF) * bd + tid];
          const float2 pk = P[(r + kSeg32) * bd + tid];
          g1 = (pb.x - pa.x) * (pk.y - pa.y) - (pb.y - pa.y) * (pk.x - pa.x) >= 0.f;
        }
      }
      const uint64_t gb0 = __ballot(g0), gb1 = __ballot(g1);
      if (fill) {
        ori = orient ? obits : (uint32_t)((gb0 >> seg0) & 0xFFFFu) | ((uint32_t)((gb1 >> seg0) & 0xFFFFu) << kSeg32);
        ori_prov = ori;
      }
      int dm = cand >= 0 ? D : 0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) dm = max(dm, __shfl_xor(dm, off));
      dmax_w = dm;
    }
    if (__ballot(r == 0 && (cand >= 0 || has_staged || in_flight)) == 0ull && exhausted) {
      if (esc_pend && r == 0) {
        EscEntry e;
        e.item = esc_item;
        e.t = (int16_t)esc_te;
        e.from_x0 = esc_te == 0 ? 1 : 0;
        e.pad = 0;
        A.esc[esc_i] = e;
      }
      break;
    }

    // ---- 2. claim the next candidate of segments that need one and issue its loads
    {
      const uint64_t want = __ballot(need_next && r == 0 && !exhausted);
      const int nwant = __popcll(want);
      if (nwant > 0) {
        const int rank = __popcll(want & ((1ull << seg0) - 1ull));
        int p = -1, given = 0;
        for (int k = 0; k < 3 && given < nwant; ++k) {
          if (cur_left == 0) {
            if (no_more) break;
            const int cur = __hip_atomic_load(&A.counters[kCntNext], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int req = min(chunk, max(nwant - given, max(items - cur, 0) / nwaves));
            int base = 0;
            if (lane == 0) base = atomicAdd(&A.counters[kCntNext], req);
            base = __shfl(base, 0);
            cur_base = base;
            cur_left = min(max(items - base, 0), req);
            if (base + req >= items) no_more = true;
          }
          const int m = min(nwant - given, cur_left);
          if (need_next && rank >= given && rank < given + m) p = cur_base + (rank - given);
          cur_base += m;
          cur_left -= m;
          given += m;
        }
        exhausted = no_more && cur_left == 0;
        if (need_next) {
          need_next = false;
          if (p >= 0) {
            in_flight = true;
            pf_t0 = 0;
            if (A.resume == 2) {  // a work item is a handed-on candidate
              const EscEntry e = A.mig_in[p];
              p = e.item;
              pf_t0 = e.t;
            }
            pf_p = p;
            pf_c = A.perm[p];
            pf_meta = reinterpret_cast<const uint32_t*>(A.meta)[p];
            pf_cf = reinterpret_cast<const float*>(A.cf + p)[r];
            // rows beyond the candidate's are loaded but not used (the record
            // arrays have J rows)
            const int s0 = min(r, J - 1), s1 = min(r + kSeg32, J - 1);
            pf_q0 = A.df[(size_t)s0 * Bs + p];
            pf_q1 = A.df[(size_t)s1 * Bs + p];
            if (A.resume == 2) {
              // its column and error bounds when it was handed on
              pf_w0 = A.esc_pos[(size_t)p * J + s0];
              pf_w1 = A.esc_pos[(size_t)p * J + s1];
              pf_e0 = A.mig_err[(size_t)p * J + s0];
              pf_e1 = A.mig_err[(size_t)p * J + s1];
            } else {
              pf_w0 = A.x0s[(size_t)s0 * Bs + p];
              pf_w1 = A.x0s[(size_t)s1 * Bs + p];
            }
          }
        }
      }
    }

    // ---- 3. one pass: lane r computes step t
    const float4* C = Ct + cpar * DMAX;
    const int t = t0 - 1 + r;
    const bool comp = cand >= 0 && !force64 && t < T && !(r == 0 && fresh);
    const uint32_t side = r == 0 ? ori_prov : ori;
    int ev = kE32None, ev_s = 0;
    if (__ballot(cand >= 0 && !force64) != 0ull) {
      if (comp) {
        const float2 cs = tab_lds ? tab[t] : A.cs32[t];
        P[D * bd + tid] = make_float2(fmaf(cs.x, vx, fmaf(-cs.y, vy, px)), fmaf(cs.y, vx, fmaf(cs.x, vy, py)));
        E[D * bd + tid] = bound_up(U);
      }
#pragma unroll
      for (int s = 0; s < DMAX; ++s) {
        if (s < dmax_w) {
          const bool act = comp && s < D && ev == kE32None;
          float2 val = P[s * bd + tid];
          uint16_t vb = E[s * bd + tid];
          float bx = 0.f, by = 0.f, ox = 0.f, oy = 0.f, h = 0.f, Eab = 0.f, rd = 0.f, R = 0.f;
          bool bK = false, lock = false, deg = false;
          bool left = false;
          if (act) {
            const float4 q = C[s];
            const uint32_t sl = __float_as_uint(q.w);
            const int a = sl & 0xFF, b = (sl >> 8) & 0xFF;
            const float2 pa = P[a * bd + tid];
            const float2 pb = P[b * bd + tid];
            const float dx = pb.x - pa.x, dy = pb.y - pa.y;
            const float d2 = fmaf(dy, dy, dx * dx);
            const float S = q.x, Dm = q.y;
            const float K = (S - d2) * (d2 - Dm);
            rd = rsq(d2);
            const float inv = rd * rd;
            const float Kp = fmaxf(K, 1e-30f);
            const float rK = rsq(Kp);
            const float sK = Kp * rK;
            const float be = sK * (0.5f * inv);
            const float al = fmaf(q.z, inv, 0.5f);
            bx = fmaf(al, dx, pa.x);
            by = fmaf(al, dy, pa.y);
            ox = -be * dy;
            oy = be * dx;
            left = (side >> s) & 1u;
            const float sgn = left ? 1.f : -1.f;
            val = make_float2(fmaf(sgn, ox, bx), fmaf(sgn, oy, by));
            P[s * bd + tid] = val;
            lock = K < 0.f;
            if ((MODE & 1) == 0) {
              const float Ea = bound_f(E[a * bd + tid]);
              const float Eb = bound_f(E[b * bd + tid]);
              Eab = Ea + Eb;
              const float d = d2 * rd;
              h = 0.5f * sK * rd;
              const float sensK = 4.f * d * fabsf(fmaf(0.5f, S + Dm, -d2));
              // as in the step-by-step pass: K's own evaluation error and the
              // rounding of this placement
              const float kthr = fmaf(sensK, Eab, fmaf(2.5f * uu, (S + d2) * (d2 + Dm), KB));
              bK = (fabsf(K) < kthr) | (d2 < CD);
              R = fmaf(uu, fabsf(pa.x) + fabsf(pa.y), U2);
              const float A2 = 0.5f * (S - Dm) * rK;  // 2 ra rb / sqrt(K)
              vb = bound_up(A2 * (Eab + R));
              E[s * bd + tid] = vb;
            } else {
              deg = d2 <= DG;
            }
          }
          // the previous step's position of this joint and its bound, from the left
          // neighbour
          const float qx = row_prev_f(val.x), qy = row_prev_f(val.y);
          const float Ep = (MODE & 1) == 0 ? bound_f((uint16_t)row_prev_i((int)vb)) : 0.f;
          if (act && r > 0) {
            const float sg = fmaf(qx - bx, ox, (qy - by) * oy);
            const bool rule_left = sg >= 0.f;
            if ((MODE & 1) == 0) {
              const float mthr = fmaf(Eab, fmaf(TS, rd, 1.f), EB + Ep + R);
              const bool band = bK | (!orient && fabsf(sg) < mthr * h);
              ev = band ? kE32Band : lock ? kE32Lock : (!orient && rule_left != left) ? kE32Side : kE32None;
            } else {
              ev = deg ? kE32Degenerate : lock ? kE32Lock : (!orient && rule_left != left) ? kE32Side : kE32None;
            }
            ev_s = s;
          }
        }
      }
    }

    // ---- 4. the next candidate's records, loaded during the pass, into LDS
    if (in_flight) {
      const int mD = pf_meta & 0xFF, mn = (pf_meta >> 8) & 0xFF;
      float4* Cn = Ct + (cpar ^ 1) * DMAX;
      if (r < mD) Cn[r] = make_float4(pf_q0.S, pf_q0.Dm, pf_q0.Kc, __uint_as_float(pf_q0.slots));
      if (r + kSeg32 < mD) Cn[r + kSeg32] = make_float4(pf_q1.S, pf_q1.Dm, pf_q1.Kc, __uint_as_float(pf_q1.slots));
      if (r < mn) PN[r] = pf_w0;
      if (r + kSeg32 < mn) PN[r + kSeg32] = pf_w1;
      if (A.resume == 2) {
        if (r < mn) EN[r] = pf_e0;
        if (r + kSeg32 < mn) EN[r + kSeg32] = pf_e1;
      }
      CFN[r] = pf_cf;
      if (r == 0) {
        MCN[0] = (int)pf_meta;
        MCN[1] = pf_c;
        MCN[2] = pf_p;
        MCN[3] = pf_t0;
      }
      in_flight = false;
      has_staged = true;
    }

    // ---- 5. the segment's first event, in step order
    const uint64_t evb = __ballot(comp && r > 0 && ev != kE32None);
    const uint32_t segm = (uint32_t)(evb >> seg0) & 0xFFFFu;
    const int f = segm ? __ffs(segm) - 1 : kSeg32;
    const int info = __shfl(ev | (ev_s << 8), seg0 + (f < kSeg32 ? f : 0));
    int kind = f < kSeg32 ? (info & 0xFF) : kE32None;
    int te = t0 - 1 + f;
    // the sides of each decided step that ends a chunk of a path row (the lanes
    // before the segment's first event), for the chunked path pass
    if (A.side_ck != nullptr && comp && r > 0 && r < f && t + 1 < T && ((t + 1) & (kPathChunk - 1)) == 0)
      A.side_ck[(size_t)cand * A.ck_n + (t + 1) / kPathChunk] = side;
    if (cand >= 0 && force64) {  // links outside the solve order: to FP64 at t = 0
      kind = kE32Band;
      te = 0;
    }
    if (cand >= 0) {
      bool done = false;
      if (kind == kE32None) {
        const int next = t0 + (kSeg32 - 1);
        if (next >= T) {
          if (r == 0) {
            A.status[cand] = 0;
            A.fail_step[cand] = -1;
            if (A.esc_step) A.esc_step[cand] = -1;
          }
          done = true;
        } else {
          t0 = next;
          ori_prov = ori;
          fresh = false;
          restarts = 0;
        }
      } else if (kind == kE32Side) {
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
          if (r == 0) A.status[cand] = kPending;
          done = true;
        }
      } else if (kind == kE32Band) {
        // to FP64 at step te from the positions of step te - 1 (lane f - 1), stored
        // at the candidate's own dump row (as every hand-over dump is); at te = 0 the
        // FP64 pass starts from the reference positions
        if (te > 0 && r == f - 1) {
          float2* dump = A.esc_pos + (size_t)item * J;
          for (int sl = 0; sl < n; ++sl) dump[sl] = P[sl * bd + tid];
        }
        if (r == 0) {
          if (A.esc_step) A.esc_step[cand] = (int16_t)te;
          if (esc_pend) {
            EscEntry e;
            e.item = esc_item;
            e.t = (int16_t)esc_te;
            e.from_x0 = esc_te == 0 ? 1 : 0;
            e.pad = 0;
            A.esc[esc_i] = e;
          }
          esc_i = atomicAdd(A.esc_cnt, 1);  // read at the next hand-over or at the end
          esc_pend = true;
          esc_item = item;
          esc_te = te;
        }
        done = true;
      } else {
        if (r == 0) {
          A.status[cand] = (uint8_t)kind;
          A.fail_step[cand] = (int16_t)te;
          if (A.esc_step) A.esc_step[cand] = -1;
        }
        done = true;
      }
      if (done) cand = -1;
    }
  }
}

template <int DMAX, int MODE>
void launch_par32_one(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  const int bd = cfg.waves * kWave;
  hipLaunchKernelGGL((simpar32_kernel<DMAX, MODE>), dim3(cfg.grid), dim3(bd), par32_lds_bytes<DMAX>(a.nslot, bd, a.T),
                     st, a);
}

template <int MODE>
hipError_t dispatch_par32(const SimArgs& a, const LaunchCfg& cfg, hipStream_t st) {
  if (a.T > kTableLds && (MODE & 2) == 0) return dispatch_par32<MODE | 2>(a, cfg, st);
  switch (sim32_dmax(a.J)) {
    case 5: launch_par32_one<5, MODE>(a, cfg, st); break;
    case 11: launch_par32_one<11, MODE>(a, cfg, st); break;
    case 18: launch_par32_one<18, MODE>(a, cfg, st); break;
    default: launch_par32_one<30, MODE>(a, cfg, st); break;
  }
  return hipGetLastError();
}

template <int DMAX, int MODE>
int occ_par32(int J, int waves, int T) {
  int nb = 0;
  const int lds = (int)par32_lds_bytes<DMAX>(J, waves * kWave, T);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, simpar32_kernel<DMAX, MODE>, waves * kWave, lds) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <int MODE>
int occ_par32_d(int J, int waves, int T) {
  switch (sim32_dmax(J)) {
    case 5: return occ_par32<5, MODE>(J, waves, T);
    case 11: return occ_par32<11, MODE>(J, waves, T);
    case 18: return occ_par32<18, MODE>(J, waves, T);
    default: return occ_par32<30, MODE>(J, waves, T);
  }
}

}  // namespace

int sim32_dmax(int J) {
  // solve-order length is at most J - 2 (the pivot and the tip are not placed)
  if (J <= 7) return 5;
  if (J <= 13) return 11;
  if (J <= 20) return 18;
  return 30;
}

int sim32_lds_bytes(int nslot, int waves, int T) {
  return nslot * waves * kWave * (int)(sizeof(float2) + sizeof(uint16_t)) +
         (T <= kTableLds ? T * (int)sizeof(float2) : 0);
}

hipError_t launch_sim32(const SimArgs& a, int mode, const LaunchCfg& cfg, hipStream_t st) {
  switch (mode) {
    case 0: return dispatch<0>(a, cfg, st);
    case 1: return dispatch<1>(a, cfg, st);
    case 4: return dispatch<4>(a, cfg, st);
    case 8: return dispatch<8>(a, cfg, st);
    case 9: return dispatch<9>(a, cfg, st);
    default: return dispatch<12>(a, cfg, st);
  }
}

template <int MODE>
int occ_d(int d, int waves, int lds) {
  switch (d) {
    case 5: return occ<5, MODE>(waves, lds);
    case 11: return occ<11, MODE>(waves, lds);
    case 18: return occ<18, MODE>(waves, lds);
    default: return occ<30, MODE>(waves, lds);
  }
}

int sim32_blocks_per_cu(int J, int mode, int T, int waves, int lds) {
  const int d = sim32_dmax(J);
  // mode 4 (recording sides) only with escalation
  const int m = (mode & 13) | (T > kTableLds ? 2 : 0);
  switch (m) {
    case 0: return occ_d<0>(d, waves, lds);
    case 1: return occ_d<1>(d, waves, lds);
    case 2: return occ_d<2>(d, waves, lds);
    case 3: return occ_d<3>(d, waves, lds);
    case 4: return occ_d<4>(d, waves, lds);
    case 6: return occ_d<6>(d, waves, lds);
    case 8: return occ_d<8>(d, waves, lds);
    case 9: return occ_d<9>(d, waves, lds);
    case 10: return occ_d<10>(d, waves, lds);
    case 11: return occ_d<11>(d, waves, lds);
    case 12: return occ_d<12>(d, waves, lds);
    default: return occ_d<14>(d, waves, lds);
  }
}

hipError_t launch_sim32_par(const SimArgs& a, int mode, const LaunchCfg& cfg, hipStream_t st) {
  return (mode & 1) == 0 ? dispatch_par32<0>(a, cfg, st) : dispatch_par32<1>(a, cfg, st);
}

int sim32_par_blocks_per_cu(int J, int mode, int T, int waves) {
  const int m = (mode & 1) | (T > kTableLds ? 2 : 0);
  switch (m) {
    case 0: return occ_par32_d<0>(J, waves, T);
    case 1: return occ_par32_d<1>(J, waves, T);
    case 2: return occ_par32_d<2>(J, waves, T);
    default: return occ_par32_d<3>(J, waves, T);
  }
}

}  // namespace links
