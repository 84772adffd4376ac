// normalize.hip -- path normalisation; FP32 paths in and out, moments and
// rotations evaluated in FP64.  PCA mode: four paths per wave (16 lanes each);
// DIAMETER mode: one wave per path.
//
// DIAMETER mode is the paper's rule (Methodology, "Dataset Curation &
// Processing"): find the longest chord of the path, turn it onto +x, scale it to
// length 1 and centre the bounding box at (0.5, 0.5).  PCA mode is the centroid /
// RMS-radius / principal-axis variant: subtract the centroid, divide by the RMS
// radius, turn the principal axis of the covariance onto +x and pick its sign so
// that the third moment along +x is positive.
//
// Sums are taken relative to the first point so that a small path far from the
// origin keeps its relative accuracy.
#include "common.h"
#include "kernels.h"

namespace links {

namespace {

constexpr int kNormWaves = 4;

__device__ __forceinline__ float wsum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ float wmin(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float wmax(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wsumd(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wmind(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wmaxd(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wsumi(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__global__ void __launch_bounds__(kNormWaves * kWave) normalize_kernel(const float* paths, int32_t P,
                                                                     const int32_t* count, int32_t T,
                                                                     int32_t mode, float* out, float* xform) {
  if (count) P = min(P, *count);
  extern __shared__ float2 pts_all[];  // [kNormWaves][T]
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  float2* pts = pts_all + (size_t)w * T;
  const int waves_total = gridDim.x * kNormWaves;
  for (int p = blockIdx.x * kNormWaves + w; p < P; p += waves_total) {
    const float2* src = reinterpret_cast<const float2*>(paths) + (size_t)p * T;
    float2* dst = reinterpret_cast<float2*>(out) + (size_t)p * T;
    const float2 p0 = src[0];
    for (int i = lane; i < T; i += kWave) pts[i] = src[i];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // coordinates relative to the first point, exact in FP64
    const double ox = p0.x, oy = p0.y;
    auto X = [&](int i) { return (double)pts[i].x - ox; };
    auto Y = [&](int i) { return (double)pts[i].y - oy; };
    float xf[5];
    if (mode == 0) {
      // ---- centroid, RMS radius, principal axis (moments accumulated in FP64: the
      // axis angle is ill-conditioned when the two eigenvalues are close)
      double sx = 0.0, sy = 0.0;
      for (int i = lane; i < T; i += kWave) {
        sx += X(i);
        sy += Y(i);
      }
      const double mx = wsumd(sx) / T, my = wsumd(sy) / T;
      double ss = 0.0;
      for (int i = lane; i < T; i += kWave) {
        const double qx = X(i) - mx, qy = Y(i) - my;
        ss += qx * qx + qy * qy;
      }
      const double s = sqrt(wsumd(ss) / T);
      const double cx = ox + mx, cy = oy + my;
      if (!(s >= 1e-12)) {
        for (int i = lane; i < T; i += kWave) dst[i] = make_float2(0.f, 0.f);
        xf[0] = (float)cx; xf[1] = (float)cy; xf[2] = 0.f; xf[3] = 0.f; xf[4] = 1.f;
      } else {
        double axx = 0.0, axy = 0.0, ayy = 0.0;
        for (int i = lane; i < T; i += kWave) {
          const double qx = (X(i) - mx) / s, qy = (Y(i) - my) / s;
          axx += qx * qx;
          axy += qx * qy;
          ayy += qy * qy;
        }
        const double cxx = wsumd(axx) / T, cxy = wsumd(axy) / T, cyy = wsumd(ayy) / T;
        const double dxy = cxx - cyy;
        const double gap = sqrt(dxy * dxy + 4.0 * cxy * cxy);
        int flags = 0;
        double phi = 0.5 * atan2(2.0 * cxy, dxy);
        if (gap < 1e-4 * (cxx + cyy)) {
          phi = 0.0;
          flags |= 2;
        }
        const double c = cos(phi), sn = sin(phi);
        double m3 = 0.0;
        for (int i = lane; i < T; i += kWave) {
          const double qx = (X(i) - mx) / s, qy = (Y(i) - my) / s;
          const double rx = c * qx + sn * qy;
          m3 += rx * rx * rx;
        }
        m3 = wsumd(m3);
        double sign = 1.0;
        if (fabs(m3) < 1e-6 * T) {
          flags |= 4;
        } else if (m3 < 0.0) {
          sign = -1.0;
          phi += 3.14159265358979323846;
        }
        for (int i = lane; i < T; i += kWave) {
          const double qx = (X(i) - mx) / s, qy = (Y(i) - my) / s;
          dst[i] = make_float2((float)(sign * (c * qx + sn * qy)), (float)(sign * (-sn * qx + c * qy)));
        }
        xf[0] = (float)cx; xf[1] = (float)cy; xf[2] = (float)s; xf[3] = (float)phi; xf[4] = (float)flags;
      }
    } else {
      // ---- longest chord: first pair (i < j) in lexicographic order
      float best = -1.f;
      int bi = 0, bj = 0;
      for (int i = lane; i < T; i += kWave) {
        const float2 a = pts[i];
        for (int j = i + 1; j < T; ++j) {
          const float dx = pts[j].x - a.x, dy = pts[j].y - a.y;
          const float d2 = fmaf(dy, dy, dx * dx);
          if (d2 > best) {
            best = d2;
            bi = i;
            bj = j;
          }
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const float ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o), oj = __shfl_xor(bj, o);
        if (ob > best || (ob == best && (oi < bi || (oi == bi && oj < bj)))) {
          best = ob;
          bi = oi;
          bj = oj;
        }
      }
      int flags = 0;
      if (!(best > 0.f) || !(sqrtf(best) >= 1e-12f)) {
        for (int i = lane; i < T; i += kWave) dst[i] = make_float2(0.f, 0.f);
        xf[0] = p0.x; xf[1] = p0.y; xf[2] = 0.f; xf[3] = 0.f; xf[4] = 1.f;
      } else {
        const float lim = (1.f - 1e-6f) * best;
        int ties = 0;
        for (int i = lane; i < T; i += kWave) {
          const float2 a = pts[i];
          for (int j = i + 1; j < T; ++j) {
            const float dx = pts[j].x - a.x, dy = pts[j].y - a.y;
            if (fmaf(dy, dy, dx * dx) >= lim && !(i == bi && j == bj)) ties++;
          }
        }
        if (wsumi(ties) > 0) flags |= 8;
        const double ax = X(bi), ay = Y(bi);
        const double ux = X(bj) - ax, uy = Y(bj) - ay;
        const double Dl = sqrt(ux * ux + uy * uy);
        const double phi = atan2(uy, ux);
        const double c = cos(phi), sn = sin(phi);
        double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
        for (int i = lane; i < T; i += kWave) {
          const double qx = X(i) - ax, qy = Y(i) - ay;
          const double rx = (c * qx + sn * qy) / Dl, ry = (-sn * qx + c * qy) / Dl;
          xmin = fmin(xmin, rx); xmax = fmax(xmax, rx);
          ymin = fmin(ymin, ry); ymax = fmax(ymax, ry);
        }
        xmin = wmind(xmin); xmax = wmaxd(xmax); ymin = wmind(ymin); ymax = wmaxd(ymax);
        const double mx = 0.5 * (xmin + xmax), my = 0.5 * (ymin + ymax);
        for (int i = lane; i < T; i += kWave) {
          const double qx = X(i) - ax, qy = Y(i) - ay;
          const double rx = (c * qx + sn * qy) / Dl, ry = (-sn * qx + c * qy) / Dl;
          dst[i] = make_float2((float)(rx - mx + 0.5), (float)(ry - my + 0.5));
        }
        xf[0] = (float)(ox + ax + Dl * (c * mx - sn * my));
        xf[1] = (float)(oy + ay + Dl * (sn * mx + c * my));
        xf[2] = (float)Dl; xf[3] = (float)phi; xf[4] = (float)flags;
      }
    }
    if (lane < 5) {
      const float v = lane == 0 ? xf[0] : lane == 1 ? xf[1] : lane == 2 ? xf[2] : lane == 3 ? xf[3] : xf[4];
      xform[(size_t)p * 5 + lane] = v;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// PCA mode, a 16-lane group per path (four paths per wave): mean, then the
// second moments about it in one pass, the third moment along the principal axis,
// and the output; every division by the RMS radius is a multiplication by its
// reciprocal.
constexpr int kPcaLanes = 16;

__device__ __forceinline__ double gsumd(double v) {
#pragma unroll
  for (int o = kPcaLanes / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__global__ void __launch_bounds__(kNormWaves * kWave) pca_kernel(const float* paths, int32_t P, const int32_t* count,
                                                                int32_t T, float* out, float* xform) {
  if (count) P = min(P, *count);
  extern __shared__ float2 pts_all[];  // [kNormWaves * 4][T]
  const int g = threadIdx.x / kPcaLanes;  // group of the workgroup
  const int l = threadIdx.x & (kPcaLanes - 1);
  float2* pts = pts_all + (size_t)g * T;
  const int groups_total = gridDim.x * (blockDim.x / kPcaLanes);
  // every group of a wave runs the same number of iterations (uniform shuffles)
  const int iters = (P + groups_total - 1) / groups_total;
  for (int k = 0; k < iters; ++k) {
    const int p = (k * gridDim.x + blockIdx.x) * (blockDim.x / kPcaLanes) + g;
    const bool live = p < P;
    const float2* src = reinterpret_cast<const float2*>(paths) + (size_t)(live ? p : 0) * T;
    float2* dst = reinterpret_cast<float2*>(out) + (size_t)p * T;
    const float2 p0 = src[0];
    for (int i = l; i < T; i += kPcaLanes) pts[i] = src[i];
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the group's LDS writes before its reads
    asm volatile("" ::: "memory");
    const double ox = p0.x, oy = p0.y;
    double sx = 0.0, sy = 0.0;
    for (int i = l; i < T; i += kPcaLanes) {
      sx += (double)pts[i].x - ox;
      sy += (double)pts[i].y - oy;
    }
    const double mx = gsumd(sx) / T, my = gsumd(sy) / T;
    double axx = 0.0, axy = 0.0, ayy = 0.0;
    for (int i = l; i < T; i += kPcaLanes) {
      const double qx = ((double)pts[i].x - ox) - mx, qy = ((double)pts[i].y - oy) - my;
      axx += qx * qx;
      axy += qx * qy;
      ayy += qy * qy;
    }
    axx = gsumd(axx);
    axy = gsumd(axy);
    ayy = gsumd(ayy);
    const double s = sqrt((axx + ayy) / T);
    const double cx = ox + mx, cy = oy + my;
    float xf[5];
    if (!(s >= 1e-12)) {
      if (live)
        for (int i = l; i < T; i += kPcaLanes) dst[i] = make_float2(0.f, 0.f);
      xf[0] = (float)cx;
      xf[1] = (float)cy;
      xf[2] = 0.f;
      xf[3] = 0.f;
      xf[4] = 1.f;
    } else {
      const double is = 1.0 / s;
      const double norm = is * is / T;  // covariance of the scaled path
      const double cxx = axx * norm, cxy = axy * norm, cyy = ayy * norm;
      const double dxy = cxx - cyy;
      const double gap = sqrt(dxy * dxy + 4.0 * cxy * cxy);
      int flags = 0;
      double phi = 0.5 * atan2(2.0 * cxy, dxy);
      if (gap < 1e-4 * (cxx + cyy)) {
        phi = 0.0;
        flags |= 2;
      }
      const double c = cos(phi), sn = sin(phi);
      double m3 = 0.0;
      for (int i = l; i < T; i += kPcaLanes) {
        const double qx = (((double)pts[i].x - ox) - mx) * is, qy = (((double)pts[i].y - oy) - my) * is;
        const double rx = c * qx + sn * qy;
        m3 += rx * rx * rx;
      }
      m3 = gsumd(m3);
      double sign = 1.0;
      if (fabs(m3) < 1e-6 * T) {
        flags |= 4;
      } else if (m3 < 0.0) {
        sign = -1.0;
        phi += 3.14159265358979323846;
      }
      const double a = sign * c, b = sign * sn;
      if (live)
        for (int i = l; i < T; i += kPcaLanes) {
          const double qx = (((double)pts[i].x - ox) - mx) * is, qy = (((double)pts[i].y - oy) - my) * is;
          dst[i] = make_float2((float)(a * qx + b * qy), (float)(-b * qx + a * qy));
        }
      xf[0] = (float)cx;
      xf[1] = (float)cy;
      xf[2] = (float)s;
      xf[3] = (float)phi;
      xf[4] = (float)flags;
    }
    if (live && l < 5) {
      const float v = l == 0 ? xf[0] : l == 1 ? xf[1] : l == 2 ? xf[2] : l == 3 ? xf[3] : xf[4];
      xform[(size_t)p * 5 + l] = v;
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);  // this path's reads before the next path's writes
    asm volatile("" ::: "memory");
  }
}

}  // namespace

hipError_t launch_normalize(const float* paths, int32_t P, const int32_t* count, int32_t T, int32_t mode,
                            float* out, float* xform, hipStream_t st) {
  if (P <= 0) return hipSuccess;
  if (mode == 0 && T <= 512) {  // 16 paths of T points in a workgroup's LDS (64 KiB at most)
    const int per_block = kNormWaves * kWave / kPcaLanes;
    int blocks = (P + per_block - 1) / per_block;
    if (blocks > 4096) blocks = 4096;
    const size_t lds = (size_t)per_block * T * sizeof(float2);
    hipLaunchKernelGGL(pca_kernel, dim3(blocks), dim3(kNormWaves * kWave), lds, st, paths, P, count, T, out, xform);
    return hipGetLastError();
  }
  int blocks = (P + kNormWaves - 1) / kNormWaves;
  if (blocks > 4096) blocks = 4096;
  size_t lds = (size_t)kNormWaves * T * sizeof(float2);
  hipLaunchKernelGGL(normalize_kernel, dim3(blocks), dim3(kNormWaves * kWave), lds, st, paths, P, count, T, mode,
                     out, xform);
  return hipGetLastError();
}

}  // namespace links
