// serve.hip -- serving support: one kernel per tick gathers the candidates of
// several requests, each stored in the server's byte ring at its own joint stride,
// into the tick's batch of the server's widest stride (the layout links_simulate
// reads), so that a request occupies the bytes of its own layout and a tick is
// one gather and one simulation (a replayed graph) whatever the requests in it.
#include "common.h"
#include "kernels.h"

namespace links {

namespace {

constexpr int kGatherBlock = 256;

__device__ __forceinline__ size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

// Byte layout of a request block of `size` candidates at stride J: x0 [size][J][2]
// f64, adj [size][J] u32, fixed [size] u32, n [size] u8, motor [size][2] u8, each
// part starting on a 16-byte boundary.
struct BlockParts {
  size_t x0, adj, fixed, n, motor;
};

__device__ __forceinline__ BlockParts parts_of(int64_t size, int J) {
  BlockParts p;
  p.x0 = 0;
  p.adj = p.x0 + align16((size_t)size * J * 16);
  p.fixed = p.adj + align16((size_t)size * J * 4);
  p.n = p.fixed + align16((size_t)size * 4);
  p.motor = p.n + align16((size_t)size);
  return p;
}

// One thread per (row, joint) of the output batch: row k = t / J, joint j = t % J,
// so consecutive threads write consecutive adj words and x0 pairs.
__global__ void __launch_bounds__(kGatherBlock) gather_kernel(const uint8_t* buf, const links_piece* pieces,
                                                               int32_t npieces, int32_t count, int32_t rows,
                                                               int32_t J, uint8_t* n, uint32_t* adj, uint32_t* fixed,
                                                               uint8_t* motor, double* x0) {
  const int64_t t = (int64_t)blockIdx.x * kGatherBlock + threadIdx.x;
  const int64_t k = t / J;
  const int j = (int)(t - k * J);
  if (k >= rows) return;
  if (k >= count) {  // a row past the tick's candidates: no joints, so never simulated
    if (j == 0) n[k] = 0;
    return;
  }
  // the piece holding row k: the last one whose first row is at most k
  int lo = 0, hi = npieces - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pieces[mid].dst <= k) lo = mid;
    else hi = mid - 1;
  }
  const links_piece pc = pieces[lo];
  const int64_t i = pc.first + (k - pc.dst);  // candidate index within its request
  const int Jr = pc.J;
  if (Jr < 1 || Jr > J || i < 0 || i >= pc.size) {  // a malformed piece: the row stays empty
    if (j == 0) n[k] = 0;
    return;
  }
  const BlockParts bp = parts_of(pc.size, Jr);
  const uint8_t* blk = buf + pc.src;
  if (j == 0) {
    // more joints than the request's stride: malformed at that stride (BAD_MECH
    // there), so no joints here either
    const uint8_t nk = blk[bp.n + i];
    n[k] = nk > Jr ? 0 : nk;
    fixed[k] = reinterpret_cast<const uint32_t*>(blk + bp.fixed)[i];
    motor[2 * k] = blk[bp.motor + 2 * i];
    motor[2 * k + 1] = blk[bp.motor + 2 * i + 1];
  }
  const bool in = j < Jr;
  adj[k * J + j] = in ? reinterpret_cast<const uint32_t*>(blk + bp.adj)[i * Jr + j] : 0u;
  reinterpret_cast<double2*>(x0)[k * J + j] =
      in ? reinterpret_cast<const double2*>(blk + bp.x0)[i * Jr + j] : make_double2(0.0, 0.0);
}

}  // namespace

hipError_t launch_gather(const uint8_t* buf, const links_piece* pieces, int32_t npieces, int32_t count,
                         int32_t rows, int32_t J, uint8_t* n, uint32_t* adj, uint32_t* fixed, uint8_t* motor,
                         double* x0, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int64_t blocks = ((int64_t)rows * J + kGatherBlock - 1) / kGatherBlock;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)blocks), dim3(kGatherBlock), 0, st, buf, pieces, npieces, count, rows, J,
                     n, adj, fixed, motor, x0);
  return hipGetLastError();
}

}  // namespace links
