// normalize.hip -- path normalisation, one wave (64 lanes) per path, FP32.
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
    for (int i = lane; i < T; i += kWave) {
      const float2 q = src[i];
      pts[i] = make_float2(q.x - p0.x, q.y - p0.y);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    float xf[5];
    if (mode == 0) {
      // ---- centroid, RMS radius, principal axis
      float sx = 0.f, sy = 0.f;
      for (int i = lane; i < T; i += kWave) {
        sx += pts[i].x;
        sy += pts[i].y;
      }
      const float mx = wsum(sx) / T, my = wsum(sy) / T;
      float ss = 0.f;
      for (int i = lane; i < T; i += kWave) {
        const float qx = pts[i].x - mx, qy = pts[i].y - my;
        ss = fmaf(qx, qx, fmaf(qy, qy, ss));
      }
      const float s = sqrtf(wsum(ss) / T);
      const float cx = p0.x + mx, cy = p0.y + my;
      if (!(s >= 1e-12f)) {
        for (int i = lane; i < T; i += kWave) dst[i] = make_float2(0.f, 0.f);
        xf[0] = cx; xf[1] = cy; xf[2] = 0.f; xf[3] = 0.f; xf[4] = 1.f;
      } else {
        const float is = 1.f / s;
        float axx = 0.f, axy = 0.f, ayy = 0.f;
        for (int i = lane; i < T; i += kWave) {
          const float qx = (pts[i].x - mx) * is, qy = (pts[i].y - my) * is;
          axx = fmaf(qx, qx, axx);
          axy = fmaf(qx, qy, axy);
          ayy = fmaf(qy, qy, ayy);
        }
        const float cxx = wsum(axx) / T, cxy = wsum(axy) / T, cyy = wsum(ayy) / T;
        const float dxy = cxx - cyy;
        const float gap = sqrtf(fmaf(dxy, dxy, 4.f * cxy * cxy));
        int flags = 0;
        float phi = 0.5f * atan2f(2.f * cxy, dxy);
        if (gap < 1e-4f * (cxx + cyy)) {
          phi = 0.f;
          flags |= 2;
        }
        float sn, c;
        sincosf(phi, &sn, &c);
        float m3 = 0.f;
        for (int i = lane; i < T; i += kWave) {
          const float qx = (pts[i].x - mx) * is, qy = (pts[i].y - my) * is;
          const float rx = fmaf(c, qx, sn * qy);
          m3 = fmaf(rx * rx, rx, m3);
        }
        m3 = wsum(m3);
        float sign = 1.f;
        if (fabsf(m3) < 1e-6f * T) {
          flags |= 4;
        } else if (m3 < 0.f) {
          sign = -1.f;
          phi += 3.14159265358979323846f;
        }
        for (int i = lane; i < T; i += kWave) {
          const float qx = (pts[i].x - mx) * is, qy = (pts[i].y - my) * is;
          dst[i] = make_float2(sign * fmaf(c, qx, sn * qy), sign * fmaf(-sn, qx, c * qy));
        }
        xf[0] = cx; xf[1] = cy; xf[2] = s; xf[3] = phi; xf[4] = (float)flags;
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
        const float Dl = sqrtf(best);
        const float ux = pts[bj].x - pts[bi].x, uy = pts[bj].y - pts[bi].y;
        const float phi = atan2f(uy, ux);
        float sn, c;
        sincosf(phi, &sn, &c);
        const float iD = 1.f / Dl;
        const float ax = pts[bi].x, ay = pts[bi].y;
        float xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
        for (int i = lane; i < T; i += kWave) {
          const float qx = pts[i].x - ax, qy = pts[i].y - ay;
          const float rx = fmaf(c, qx, sn * qy) * iD, ry = fmaf(-sn, qx, c * qy) * iD;
          xmin = fminf(xmin, rx); xmax = fmaxf(xmax, rx);
          ymin = fminf(ymin, ry); ymax = fmaxf(ymax, ry);
        }
        xmin = wmin(xmin); xmax = wmax(xmax); ymin = wmin(ymin); ymax = wmax(ymax);
        const float mx = 0.5f * (xmin + xmax), my = 0.5f * (ymin + ymax);
        for (int i = lane; i < T; i += kWave) {
          const float qx = pts[i].x - ax, qy = pts[i].y - ay;
          const float rx = fmaf(c, qx, sn * qy) * iD, ry = fmaf(-sn, qx, c * qy) * iD;
          dst[i] = make_float2(rx - mx + 0.5f, ry - my + 0.5f);
        }
        xf[0] = p0.x + ax + Dl * (c * mx - sn * my);
        xf[1] = p0.y + ay + Dl * (sn * mx + c * my);
        xf[2] = Dl; xf[3] = phi; xf[4] = (float)flags;
      }
    }
    if (lane < 5) {
      const float v = lane == 0 ? xf[0] : lane == 1 ? xf[1] : lane == 2 ? xf[2] : lane == 3 ? xf[3] : xf[4];
      xform[(size_t)p * 5 + lane] = v;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

}  // namespace

hipError_t launch_normalize(const float* paths, int32_t P, const int32_t* count, int32_t T, int32_t mode,
                            float* out, float* xform, hipStream_t st) {
  if (P <= 0) return hipSuccess;
  int blocks = (P + kNormWaves - 1) / kNormWaves;
  if (blocks > 4096) blocks = 4096;
  size_t lds = (size_t)kNormWaves * T * sizeof(float2);
  hipLaunchKernelGGL(normalize_kernel, dim3(blocks), dim3(kNormWaves * kWave), lds, st, paths, P, count, T, mode,
                     out, xform);
  return hipGetLastError();
}

}  // namespace links
