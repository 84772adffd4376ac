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

// squared distance written as (x_p - x_q)^2 + (y_p - y_q)^2, the reference's operation order
__device__ inline double sqd(const double* p, const double* q) {
  double dx = p[0] - q[0];
  double dy = p[1] - q[1];
  return dx * dx + dy * dy;
}

constexpr int kPrepBlock = 128;

__global__ void __launch_bounds__(kPrepBlock) prep_kernel(PrepArgs A) {
  __shared__ uint32_t ord_l[kMaxJ][kPrepBlock];  // (k | a << 8 | b << 16) per entry
  __shared__ uint8_t idx_l[kMaxJ][kPrepBlock];   // solve-order index of each placed joint
  const int tid = threadIdx.x;
  const int c = blockIdx.x * blockDim.x + tid;
  if (c >= A.B) return;
  const int J = A.J;
  const int n = A.n[c];
  const uint32_t* adj = A.adj + (size_t)c * J;
  const uint32_t fixed = A.fixed[c];
  const int pivot = A.motor[2 * c], tip = A.motor[2 * c + 1];

  // ---- integer structure (same rules as links_solve_order documents)
  bool ok = n >= 3 && n <= J;
  const uint32_t live = live_mask(n);
  if (ok && (fixed & ~live)) ok = false;
  for (int i = 0; ok && i < J; i++) {
    uint32_t r = adj[i];
    if (i >= n) {
      if (r) ok = false;
      continue;
    }
    if ((r & ~live) || ((r >> i) & 1u)) {
      ok = false;
      break;
    }
    for (uint32_t m = r; m; m &= m - 1u) {
      int j = lowbit(m);
      if (!((adj[j] >> i) & 1u)) ok = false;
    }
  }
  if (ok && (pivot >= n || tip >= n || pivot == tip)) ok = false;
  if (ok && (!((fixed >> pivot) & 1u) || ((fixed >> tip) & 1u) || !((adj[pivot] >> tip) & 1u))) ok = false;

  int nd = 0, depth = 0;
  bool complete = false;
  if (ok) {
    // ---- rounds of the graphical solver
    uint32_t known = fixed | (1u << tip);
    for (;;) {
      uint32_t now = 0u;
      for (int k = 0; k < n; k++) {
        if ((known >> k) & 1u) continue;
        uint32_t kn = adj[k] & known;
        if (popc(kn) < 2) continue;
        int a = lowbit(kn);
        int b = lowbit(kn & (kn - 1u));
        ord_l[nd][tid] = (uint32_t)k | ((uint32_t)a << 8) | ((uint32_t)b << 16);
        idx_l[k][tid] = (uint8_t)nd;
        nd++;
        now |= 1u << k;
      }
      if (!now) break;
      known |= now;
      depth++;
    }
    complete = known == live;
  }

  // ---- solve-order outputs
  if (A.order) {
    int8_t* o = A.order + (size_t)c * J * 3;
    for (int s = 0; s < J; s++) {
      bool has = ok && s < nd;
      uint32_t e = has ? ord_l[s][tid] : 0u;
      o[3 * s + 0] = has ? (int8_t)(e & 0xFF) : (int8_t)-1;
      o[3 * s + 1] = has ? (int8_t)((e >> 8) & 0xFF) : (int8_t)-1;
      o[3 * s + 2] = has ? (int8_t)((e >> 16) & 0xFF) : (int8_t)-1;
    }
  }
  if (A.n_dyads) A.n_dyads[c] = ok ? (uint8_t)nd : 0;
  if (A.depth) A.depth[c] = ok ? (uint8_t)depth : 0;
  if (!A.sim) {
    A.status[c] = !ok ? 5 : (complete ? 0 : 4);
    return;
  }

  // ---- simulation records
  const double* x0 = A.x0 + (size_t)c * J * 2;
  double scale = 0.0;
  if (ok) {
    for (int i = 0; i < n; i++)
      if (!isfinite(x0[2 * i]) || !isfinite(x0[2 * i + 1])) ok = false;
  }
  int redundant = 0;
  if (ok) {
    for (int i = 0; i < n; i++)
      for (uint32_t m = adj[i] & ~((2u << i) - 1u); m; m &= m - 1u) {
        int j = lowbit(m);
        double L = sqrt(sqd(x0 + 2 * i, x0 + 2 * j));
        if (!(L > 1e-12)) ok = false;
        if (L > scale) scale = L;
        if (!(((fixed >> i) & 1u) && ((fixed >> j) & 1u))) redundant++;
      }
  }
  if (!ok) {
    A.status[c] = 5;
    A.fail_step[c] = -1;
    if (A.esc_step) A.esc_step[c] = -1;
    return;
  }
  if (!complete) {
    A.status[c] = 4;
    A.fail_step[c] = -1;
    if (A.esc_step) A.esc_step[c] = -1;
    return;
  }
  // links outside the solve order: all but the actuator arm and 2 per placed joint
  redundant -= 1 + 2 * nd;

  const int D = nd;
  auto slot_of = [&](int j) -> int {
    if (j == tip) return D;
    if ((fixed >> j) & 1u) return D + 1 + popc(fixed & ((1u << j) - 1u));
    return idx_l[j][tid];
  };
  CandMeta m;
  m.D = (uint8_t)D;
  m.n = (uint8_t)n;
  int out = A.out_joint;
  uint32_t flags = redundant > 0 ? kFlagRedundant : 0u;
  if (out < 0) out = D > 0 ? (int)(ord_l[D - 1][tid] & 0xFF) : tip;
  if (out >= n) {
    flags |= kFlagNoPath;
    m.out_slot = 0;
  } else {
    m.out_slot = (uint8_t)slot_of(out);
  }
  m.flags = (uint8_t)flags;
  A.meta[c] = m;

  const double px = x0[2 * pivot], py = x0[2 * pivot + 1];
  const double vx = x0[2 * tip] - px, vy = x0[2 * tip + 1] - py;
  const double scale2 = scale * scale;
  CandF64 cd;
  cd.px = px;
  cd.py = py;
  cd.vx = vx;
  cd.vy = vy;
  cd.scale = scale;
  cd.deg_thr = 1e-12 * scale2;
  cd.drift_thr = A.tau_drift * scale;
  cd.pad = 0.0;
  A.cd[c] = cd;

  // FP32 thresholds and error units (a computed position carries at most a few
  // ulps of its magnitude before amplification)
  const double u = 4.0 * 5.9604644775390625e-08;
  CandF32 cf;
  cf.px = (float)px;
  cf.py = (float)py;
  cf.vx = (float)vx;
  cf.vy = (float)vy;
  cf.U = (float)(u * (fabs(px) + fabs(py) + fabs(vx) + fabs(vy)));
  cf.KB = (float)(4.0 * A.eps_disc * scale2 * scale2);
  cf.CD = (float)(A.eps_disc * scale2);
  cf.EB = (float)(A.eps_branch * scale);
  cf.EP = (float)(A.path_tol * scale);
  cf.U2 = (float)(u * 2.0 * scale);
  cf.TS = (float)(2.0 * scale);
  cf.u = (float)u;
  cf.DG = (float)(1e-12 * scale2);
  cf.pad[0] = cf.pad[1] = cf.pad[2] = 0.f;
  A.cf[c] = cf;

  DyadF32* df = A.df + (size_t)c * J;
  DyadF64* dd = A.dd + (size_t)c * J;
  for (int s = 0; s < D; s++) {
    uint32_t e = ord_l[s][tid];
    int k = e & 0xFF, a = (e >> 8) & 0xFF, b = (e >> 16) & 0xFF;
    double ra2 = sqd(x0 + 2 * k, x0 + 2 * a);
    double rb2 = sqd(x0 + 2 * k, x0 + 2 * b);
    double ra = sqrt(ra2), rb = sqrt(rb2);
    double sum = ra + rb, dif = ra - rb;
    DyadF64 q;
    q.ra2 = ra2;
    q.rb2 = rb2;
    q.S = sum * sum;
    q.Dm = dif * dif;
    dd[s] = q;
    DyadF32 f;
    f.S = (float)(sum * sum);
    f.Dm = (float)(dif * dif);
    f.Kc = (float)(0.5 * (ra2 - rb2));
    f.slots = (uint32_t)slot_of(a) | ((uint32_t)slot_of(b) << 8);
    df[s] = f;
  }
  float2* xs = A.x0s + (size_t)c * J;
  uint8_t* sj = A.slot_joint + (size_t)c * J;
  for (int j = 0; j < n; j++) {
    int sl = slot_of(j);
    xs[sl] = make_float2((float)x0[2 * j], (float)x0[2 * j + 1]);
    sj[sl] = (uint8_t)j;
  }
  A.status[c] = kPending;
  atomicAdd(&A.counters[kCntHist + D], 1);
}

// Exclusive offsets of the D histogram, largest D first (one thread).
__global__ void bucket_scan_kernel(int32_t* counters, int32_t first_item) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t off = first_item;
  for (int d = kMaxJ - 1; d >= 0; d--) {
    int32_t h = counters[kCntHist + d];
    counters[kCntOff + d] = off;
    off += h;
  }
  counters[kCntItems] = off;
  counters[kCntNext] = first_item;
}

__global__ void bucket_scatter_kernel(int32_t B, const uint8_t* status, const CandMeta* meta,
                                      int32_t* counters, int32_t* perm) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= B || status[c] != kPending) return;
  int d = meta[c].D;
  int p = atomicAdd(&counters[kCntOff + d], 1);
  perm[p] = c;
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
                                                                  int32_t* index, int32_t cap) {
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
}

// Copies the staged rows of the valid candidates into the compacted output.
__global__ void gather_rows_kernel(const int32_t* index, const int32_t* total, int32_t cap,
                                   const uint4* staged, uint4* out, int32_t row_vec4) {
  int rows = min(*total, cap);
  for (int r = blockIdx.x; r < rows; r += gridDim.x) {
    const uint4* src = staged + (size_t)index[r] * row_vec4;
    uint4* dst = out + (size_t)r * row_vec4;
    for (int i = threadIdx.x; i < row_vec4; i += blockDim.x) dst[i] = src[i];
  }
}

__global__ void gather_rows_f2_kernel(const int32_t* index, const int32_t* total, int32_t cap,
                                      const float2* staged, float2* out, int32_t row) {
  int rows = min(*total, cap);
  for (int r = blockIdx.x; r < rows; r += gridDim.x) {
    const float2* src = staged + (size_t)index[r] * row;
    float2* dst = out + (size_t)r * row;
    for (int i = threadIdx.x; i < row; i += blockDim.x) dst[i] = src[i];
  }
}

}  // namespace

hipError_t launch_prep(const PrepArgs& a, hipStream_t st) {
  if (a.B <= 0) return hipSuccess;
  int grid = (a.B + kPrepBlock - 1) / kPrepBlock;
  hipLaunchKernelGGL(prep_kernel, dim3(grid), dim3(kPrepBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_bucket_sort(int32_t B, const uint8_t* status, const CandMeta* meta, int32_t* counters,
                              int32_t* perm, hipStream_t st) {
  hipLaunchKernelGGL(bucket_scan_kernel, dim3(1), dim3(64), 0, st, counters, 0);
  if (B > 0) {
    int grid = (B + 255) / 256;
    hipLaunchKernelGGL(bucket_scatter_kernel, dim3(grid), dim3(256), 0, st, B, status, meta, counters, perm);
  }
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

hipError_t launch_compact(int32_t B, const uint8_t* status, int32_t* scratch, int32_t* index, int32_t cap,
                          int32_t* total, hipStream_t st) {
  int nb = (B + kScanBlock - 1) / kScanBlock;
  if (nb == 0) {
    return launch_fill_u32(total, 1, 0u, st);
  }
  hipLaunchKernelGGL(count_valid_kernel, dim3(nb), dim3(kScanBlock), 0, st, B, status, scratch);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, st, nb, scratch, total);
  hipLaunchKernelGGL(write_index_kernel, dim3(nb), dim3(kScanBlock), 0, st, B, status, scratch, index, cap);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const int32_t* index, const int32_t* total, int32_t cap, const void* staged,
                              void* out, size_t row_bytes, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  int grid = cap < 8192 ? cap : 8192;
  if (row_bytes % 16 == 0) {
    hipLaunchKernelGGL(gather_rows_kernel, dim3(grid), dim3(128), 0, st, index, total, cap,
                       (const uint4*)staged, (uint4*)out, (int32_t)(row_bytes / 16));
  } else {
    hipLaunchKernelGGL(gather_rows_f2_kernel, dim3(grid), dim3(128), 0, st, index, total, cap,
                       (const float2*)staged, (float2*)out, (int32_t)(row_bytes / 8));
  }
  return hipGetLastError();
}

}  // namespace links
