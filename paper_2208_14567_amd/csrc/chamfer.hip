// chamfer.hip -- bidirectional chamfer distance between normalised paths and the
// retrieval searches built on it ("A Case Study of Mechanism Retrieval").
//
// CD(A, B) = mean over a in A of min over b in B of |a - b|
//          + mean over b in B of min over a in A of |a - b|
// for two paths of T points each, in FP32 from exact coordinate differences
// (no |a|^2 + |b|^2 - 2 a.b expansion, which cancels for close points).
//
// One wave compares one query with one bank path at a time.  Its 64 lanes form
// an 8 x 8 grid: lane (u, v) = (lane & 7, lane >> 3) holds the query points
// i = u + 8 r (r < NA) in registers for the whole launch and streams the bank
// points j = v + 8 s (s < NA), so each lane evaluates NA x NA of the T x T
// pairs.  Row minima (per query point) are reduced over v, column minima (per
// bank point) over u.  Indices past T - 1 repeat point T - 1: a repeated point
// leaves every minimum unchanged and is left out of the sums.
//
// Selection keeps, per wave, the kChamferKeep smallest 64-bit keys of the paths under
// the cut-off (FIRST: position then distance bits; BEST: distance bits then
// position -- distances are >= 0, so their bit patterns order like the values);
// a merge kernel combines the waves' lists with the result of earlier launches.
#include "kernels.h"

namespace links {

namespace {

constexpr uint64_t kEmptyKey = ~0ull;

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float swz_xor16(float x) {
  // ds_swizzle bit mode: and_mask 0x1F, or_mask 0, xor_mask 0x10
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x401F));
}

__device__ __forceinline__ float xor32(float x) { return __shfl_xor(x, 32); }

// Minima are taken on the bit patterns of non-negative floats (squared
// distances and +inf), which order like the values; this keeps the reductions
// free of NaN canonicalisation.
__device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

template <int CTRL>
__device__ __forceinline__ uint32_t dppu(uint32_t x) {
  return __builtin_amdgcn_update_dpp(0u, x, CTRL, 0xF, 0xF, false);
}

// all-reduce over the 8 lanes sharing v (lane bits 0..2)
__device__ __forceinline__ float min_over_u(float xf) {
  uint32_t x = __float_as_uint(xf);
  x = umin(x, dppu<0xB1>(x));   // quad_perm [1,0,3,2]: lane ^ 1
  x = umin(x, dppu<0x4E>(x));   // quad_perm [2,3,0,1]: lane ^ 2
  return __uint_as_float(umin(x, dppu<0x141>(x)));  // row_half_mirror: the other quad of the 8
}
__device__ __forceinline__ float sum_over_u(float x) {
  x = x + dpp<0xB1>(x);
  x = x + dpp<0x4E>(x);
  return x + dpp<0x141>(x);
}
// all-reduce over the 8 lanes sharing u (lane bits 3..5)
__device__ __forceinline__ float min_over_v(float xf) {
  uint32_t x = __float_as_uint(xf);
  x = umin(x, dppu<0x128>(x));  // row_ror:8: lane ^ 8 within each row of 16
  x = umin(x, (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x401F));  // lane ^ 16
  return __uint_as_float(umin(x, (uint32_t)__shfl_xor((int)x, 32)));
}
__device__ __forceinline__ float sum_over_v(float x) {
  x = x + dpp<0x128>(x);
  x = x + swz_xor16(x);
  return x + xor32(x);
}

// inserts key into the ascending list keep[0..kChamferKeep) (the largest falls off)
__device__ __forceinline__ void insert_key(uint64_t (&keep)[kChamferKeep], uint64_t key) {
#pragma unroll
  for (int i = kChamferKeep - 1; i > 0; i--) {
    const uint64_t lo = keep[i - 1];
    keep[i] = key < lo ? lo : (key < keep[i] ? key : keep[i]);
  }
  keep[0] = key < keep[0] ? key : keep[0];
}

// The same list spread over lanes 0..15 of a wave (lane i holds entry i): the
// entry below comes from the previous lane (DPP row_shr:1; lane 0 sees 0).
__device__ __forceinline__ uint64_t insert_key_lanes(uint64_t mine, uint64_t key) {
  const uint32_t lo = __builtin_amdgcn_update_dpp(0, (uint32_t)mine, 0x111, 0xF, 0xF, false);
  const uint32_t hi = __builtin_amdgcn_update_dpp(0, (uint32_t)(mine >> 32), 0x111, 0xF, 0xF, false);
  const uint64_t below = (uint64_t)hi << 32 | lo;
  return key < below ? below : (key < mine ? key : mine);
}

// EXACT: NA = ceil(T / 8), so only the last r and s can reach past T - 1.
template <int NA, bool EXACT>
__global__ __launch_bounds__(256) void chamfer_kernel(ChamferArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t q = gw / A.waves_per_query;
  if (q >= A.Q) return;  // the whole wave leaves (grid rounding)
  const int w = (int)(gw - q * A.waves_per_query);
  const int u = lane & 7, v = lane >> 3;
  const int T = A.T;

  const float2* qp = A.queries + q * T;
  float ax[NA], ay[NA];
#pragma unroll
  for (int r = 0; r < NA; r++) {
    const float2 t = qp[EXACT && r < NA - 1 ? u + 8 * r : min(u + 8 * r, T - 1)];
    ax[r] = t.x;
    ay[r] = t.y;
  }
  const float fT = (float)T;

  uint64_t keep = kEmptyKey;  // lane i < kChamferKeep: the i-th smallest key so far

  // FIRST: a query that already holds k matches from earlier rows is finished
  const bool done = A.k > 0 && A.order == kChamferFirst && A.running != nullptr &&
                    A.running[q * kChamferKeep + A.k - 1] != kEmptyKey;
  for (int64_t p = A.p_lo + w; !done && p < A.p_hi; p += A.waves_per_query) {
    const float2* bp = A.bank + p * T;
    float rmin[NA];
#pragma unroll
    for (int r = 0; r < NA; r++) rmin[r] = __builtin_inff();
    float csum = 0.f;
#pragma unroll
    for (int s = 0; s < NA; s++) {
      const int j = v + 8 * s;
      const float2 b = bp[EXACT && s < NA - 1 ? j : min(j, T - 1)];
      float cm = __builtin_inff();
#pragma unroll
      for (int r = 0; r < NA; r++) {
        const float dx = ax[r] - b.x, dy = ay[r] - b.y;
        const float d2 = fmaf(dx, dx, dy * dy);
        rmin[r] = fminf(rmin[r], d2);
        cm = fminf(cm, d2);
      }
      cm = min_over_u(cm);
      if ((EXACT && s < NA - 1) || j < T) csum += __builtin_amdgcn_sqrtf(cm);
    }
    float rsum = 0.f;
#pragma unroll
    for (int r = 0; r < NA; r++) {
      const float m = min_over_v(rmin[r]);
      if ((EXACT && r < NA - 1) || u + 8 * r < T) rsum += __builtin_amdgcn_sqrtf(m);
    }
    rsum = sum_over_u(rsum);
    csum = sum_over_v(csum);
    float cd = rsum / fT + csum / fT;
    // a non-finite point leaves +inf (or NaN) in its own minimum, so only a pair
    // of finite paths whose squared distances stay in range gets a finite CD
    if (!(cd < __builtin_inff())) cd = __builtin_nanf("");

    if (A.dist != nullptr && lane == 0) A.dist[q * A.P + p] = cd;
    if (A.k > 0 && cd < A.cutoff) {  // the same on every lane
      const uint32_t db = __float_as_uint(cd), pi = (uint32_t)p;
      const uint64_t key = A.order == kChamferFirst ? ((uint64_t)pi << 32 | db) : ((uint64_t)db << 32 | pi);
      keep = insert_key_lanes(keep, key);
      if (A.order == kChamferFirst) {
        // k hits at lower positions than any later path of this wave
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)keep, A.k - 1);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(keep >> 32), A.k - 1);
        if (((uint64_t)hi << 32 | lo) != kEmptyKey) break;
      }
    }
  }
  if (A.k > 0 && lane < kChamferKeep) A.part[(q * A.waves_per_query + w) * kChamferKeep + lane] = keep;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m) {
  const uint32_t lo = __shfl_xor((uint32_t)x, m), hi = __shfl_xor((uint32_t)(x >> 32), m);
  return (uint64_t)hi << 32 | lo;
}

// One workgroup per query: the kChamferKeep smallest keys among the waves' lists and
// the running result, written back to the running result and to idx / dist.
__global__ __launch_bounds__(256) void chamfer_merge_kernel(ChamferArgs A, uint64_t* running, int64_t* idx,
                                                            float* dist) {
  __shared__ uint64_t lists[256][kChamferKeep];
  __shared__ uint64_t wmin[4];
  const int64_t q = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint64_t keep[kChamferKeep];
#pragma unroll
  for (int i = 0; i < kChamferKeep; i++) keep[i] = kEmptyKey;
  const int64_t n = (int64_t)A.waves_per_query * kChamferKeep;
  const uint64_t* src = A.part + q * n;
  for (int64_t e = tid; e < n; e += 256) {
    const uint64_t key = src[e];
    if (key < keep[kChamferKeep - 1]) insert_key(keep, key);
  }
  if (tid < kChamferKeep) {
    const uint64_t key = running[q * kChamferKeep + tid];
    if (key < keep[kChamferKeep - 1]) insert_key(keep, key);
  }
#pragma unroll
  for (int i = 0; i < kChamferKeep; i++) lists[tid][i] = keep[i];
  __syncthreads();
  int head = 0;
  for (int r = 0; r < A.k; r++) {
    uint64_t c = head < kChamferKeep ? lists[tid][head] : kEmptyKey;
    uint64_t m = c;
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t o = shfl_xor_u64(m, off);
      m = o < m ? o : m;
    }
    if (lane == 0) wmin[wv] = m;
    __syncthreads();
    uint64_t sel = wmin[0];
#pragma unroll
    for (int i = 1; i < 4; i++) sel = wmin[i] < sel ? wmin[i] : sel;
    __syncthreads();
    if (sel != kEmptyKey && c == sel) head++;  // keys are unique
    if (tid == 0) {
      running[q * kChamferKeep + r] = sel;
      int64_t id = -1;
      float d = __builtin_nanf("");
      if (sel != kEmptyKey) {
        const uint32_t hi = (uint32_t)(sel >> 32), lo = (uint32_t)sel;
        id = A.order == kChamferFirst ? hi : lo;
        d = __uint_as_float(A.order == kChamferFirst ? lo : hi);
      }
      idx[q * A.k + r] = id;
      dist[q * A.k + r] = d;
    }
  }
}

template <int NA, bool EXACT>
hipError_t launch_na(const ChamferArgs& a, int64_t blocks, hipStream_t st) {
  hipLaunchKernelGGL((chamfer_kernel<NA, EXACT>), dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int NA, bool EXACT>
int occ_na() {
  int nb = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, chamfer_kernel<NA, EXACT>, 256, 0);
  return e == hipSuccess && nb > 0 ? nb : 1;
}

}  // namespace

// Instantiated register tiles: T = 8 NA uses the exact kernel (T = 200: NA = 25),
// other T the next larger tile with repeated points.
int chamfer_na(int T) {
  const int na = (T + 7) / 8;
  return na <= 2 ? 2 : na <= 4 ? 4 : na <= 7 ? 7 : na <= 8 ? 8 : na <= 13 ? 13 : na <= 16 ? 16 : na <= 25 ? 25 : 32;
}

#define LINKS_CHAMFER_DISPATCH(T, CALL)                     \
  do {                                                      \
    const bool ex_ = chamfer_na(T) == ((T) + 7) / 8;        \
    switch (chamfer_na(T)) {                                \
      case 2: return ex_ ? CALL(2, true) : CALL(2, false);   \
      case 4: return ex_ ? CALL(4, true) : CALL(4, false);   \
      case 7: return ex_ ? CALL(7, true) : CALL(7, false);   \
      case 8: return ex_ ? CALL(8, true) : CALL(8, false);   \
      case 13: return ex_ ? CALL(13, true) : CALL(13, false); \
      case 16: return ex_ ? CALL(16, true) : CALL(16, false); \
      case 25: return ex_ ? CALL(25, true) : CALL(25, false); \
      default: return ex_ ? CALL(32, true) : CALL(32, false); \
    }                                                       \
  } while (0)

int chamfer_blocks_per_cu(int T) {
#define LINKS_OCC(NA, EX) occ_na<NA, EX>()
  LINKS_CHAMFER_DISPATCH(T, LINKS_OCC);
#undef LINKS_OCC
}

hipError_t launch_chamfer(const ChamferArgs& a, hipStream_t st) {
  const int64_t waves = a.Q * (int64_t)a.waves_per_query;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks == 0 || a.p_hi <= a.p_lo) return hipSuccess;
#define LINKS_GO(NA, EX) launch_na<NA, EX>(a, blocks, st)
  LINKS_CHAMFER_DISPATCH(a.T, LINKS_GO);
#undef LINKS_GO
}

hipError_t launch_chamfer_merge(const ChamferArgs& a, uint64_t* running, int64_t* idx, float* dist,
                                hipStream_t st) {
  if (a.Q == 0) return hipSuccess;
  hipLaunchKernelGGL(chamfer_merge_kernel, dim3((unsigned)a.Q), dim3(256), 0, st, a, running, idx, dist);
  return hipGetLastError();
}

__global__ void chamfer_clear_kernel(uint64_t* running, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) running[i] = kEmptyKey;
}

hipError_t launch_chamfer_clear(uint64_t* running, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(chamfer_clear_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, running, n);
  return hipGetLastError();
}

}  // namespace links
