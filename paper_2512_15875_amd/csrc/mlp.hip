// Learned local preconditioner: elementwise and feature kernels.  The dense
// layers run on the offset-table GEMM engine (mlp_api.cpp); this file holds
// bias + SiLU, its backward, bias gradients, the MSE loss, Adam, and the
// tile features / tile reassembly of local vectors.
//
// Features of one tile of T = 64 consecutive entries of a local vector b
// with diagonal d = diag(H_eff) - s:  [b_tile / |b|, d_tile / sigma]  (128
// values, zero-padded past the end), sigma = mean |d| over the node (the
// scale of the local shifted operator).  The network's 64 outputs are the
// correction tile in units of |b| / sigma.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace ttn {

__device__ __forceinline__ float silu(float x) { return x / (1.0f + expf(-x)); }
__device__ __forceinline__ float dsilu(float x) {
  const float s = 1.0f / (1.0f + expf(-x));
  return s * (1.0f + x * (1.0f - s));
}

// pre[i][j] += bias[j]; post = silu(pre) (act != 0) or pre
__global__ void bias_act_kernel(float* pre, float* post, const float* bias, int n, int w, int act) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * w) return;
  const int j = (int)(e % w);
  const float v = pre[e] + bias[j];
  pre[e] = v;
  post[e] = act ? silu(v) : v;
}

// g[i][j] *= silu'(pre[i][j])
__global__ void dact_kernel(float* g, const float* pre, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < total) g[e] *= dsilu(pre[e]);
}

// db[j] = sum_i g[i][j]
__global__ void colsum_kernel(const float* g, int n, int w, float* db) {
  const int j = blockIdx.x;
  float s = 0;
  for (int i = threadIdx.x; i < n; i += 256) s += g[(int64_t)i * w + j];
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[j] = red[0];
}

// dY = 2 (Y - T) / (n * w);  loss partials (sum of squares)
__global__ void mse_kernel(const float* Y, const float* Tg, float* dY, int64_t total, double scale, double* loss) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0;
  if (e < total) {
    const double d = (double)Y[e] - (double)Tg[e];
    dY[e] = (float)(2.0 * d * scale);
    v = d * d;
  }
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] * scale);
}

__global__ void adam_kernel(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.0f - b1) * gi;
  const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// per state: |b| and sigma = mean |d|
template <typename T>
__global__ __launch_bounds__(256) void feat_scale_kernel(const T* b, const T* d, int64_t n, double* scales) {
  const int z = blockIdx.x;
  const T* bz = b + (int64_t)z * n;
  const T* dz = d + (int64_t)z * n;
  double sb = 0, sd = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    sb += (double)bz[i] * (double)bz[i];
    sd += fabs((double)dz[i]);
  }
  __shared__ double r1[256], r2[256];
  r1[threadIdx.x] = sb;
  r2[threadIdx.x] = sd;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      r1[threadIdx.x] += r1[threadIdx.x + o];
      r2[threadIdx.x] += r2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scales[2 * z] = sqrt(r1[0]);
    scales[2 * z + 1] = n > 0 ? r2[0] / (double)n : 0.0;
  }
}

// X[(z*ntiles + t)][0..64) = b/|b|, [64..128) = d/sigma
template <typename T>
__global__ void feat_kernel(const T* b, const T* d, int64_t n, int ntiles, const double* scales, float* X, int nz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)ntiles * 128;
  if (e >= per * nz) return;
  const int z = (int)(e / per);
  const int64_t r = e - (int64_t)z * per;
  const int t = (int)(r / 128), c = (int)(r - (int64_t)t * 128);
  const int64_t i = (int64_t)t * 64 + (c & 63);
  const double nb = scales[2 * z], sg = scales[2 * z + 1];
  float v = 0.0f;
  if (i < n) {
    if (c < 64) v = nb > 0 ? (float)((double)b[(int64_t)z * n + i] / nb) : 0.0f;
    else v = sg > 0 ? (float)((double)d[(int64_t)z * n + i] / sg) : 0.0f;
  }
  X[e] = v;
}

// target tiles in network units: the correction to the DIAG step,
// (y - b / d) * sigma / |b| (zero past the end and where d = 0)
template <typename T>
__global__ void target_kernel(const T* y, const T* b, const T* d, int64_t n, int ntiles, const double* scales, float* Yt,
                              int nz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)ntiles * 64;
  if (e >= per * nz) return;
  const int z = (int)(e / per);
  const int64_t i = e - (int64_t)z * per;
  const double nb = scales[2 * z], sg = scales[2 * z + 1];
  float v = 0.0f;
  if (i < n && nb > 0) {
    const int64_t o = (int64_t)z * n + i;
    const double dd = (double)d[o];
    const double yd = dd != 0.0 ? (double)b[o] / dd : 0.0;
    v = (float)(((double)y[o] - yd) * sg / nb);
  }
  Yt[e] = v;
}

// y = out * |b| / sigma (tiles back into local vectors)
template <typename T>
__global__ void untile_kernel(const float* Yn, int64_t n, int ntiles, const double* scales, T* y, int nz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nz) return;
  const int z = (int)(e / n);
  const int64_t i = e - (int64_t)z * n;
  const double nb = scales[2 * z], sg = scales[2 * z + 1];
  y[e] = (T)(sg > 0 ? (double)Yn[(int64_t)z * ntiles * 64 + i] * nb / sg : 0.0);
}

// Minimal-residual combination of two candidate solutions of (A) y = b, given
// their images Pd = A yd and Pl = A yl: per state the FP64 Gram entries and
// overlaps, then (a, c) minimising |a Pd + c Pl - b|.  c = 0 (DIAG alone,
// with its best scale) when the two images are numerically parallel or any
// sum is not finite.
template <typename T>
__global__ __launch_bounds__(256) void mr2_kernel(const T* Pd, const T* Pl, const T* b, int64_t n, double* coef) {
  const int z = blockIdx.x;
  const T* pd = Pd + (int64_t)z * n;
  const T* pl = Pl + (int64_t)z * n;
  const T* bz = b + (int64_t)z * n;
  double s[5] = {0, 0, 0, 0, 0};
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double x = (double)pd[i], y = (double)pl[i], r = (double)bz[i];
    s[0] += x * x;
    s[1] += x * y;
    s[2] += y * y;
    s[3] += x * r;
    s[4] += y * r;
  }
  __shared__ double red[5][256];
  for (int q = 0; q < 5; ++q) red[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int q = 0; q < 5; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double dd = red[0][0], dl = red[1][0], ll = red[2][0], bd = red[3][0], bl = red[4][0];
    double a = dd > 0 ? bd / dd : 1.0, c = 0.0;
    const double det = dd * ll - dl * dl;
    if (isfinite(det) && isfinite(ll) && isfinite(bl) && det > 1e-10 * dd * ll) {
      const double a2 = (bd * ll - bl * dl) / det, c2 = (bl * dd - bd * dl) / det;
      if (isfinite(a2) && isfinite(c2)) {
        a = a2;
        c = c2;
      }
    }
    if (!isfinite(a)) a = 1.0;
    coef[2 * z] = a;
    coef[2 * z + 1] = c;
  }
}

// y = a yd + c yl per state (yl not read where c = 0)
template <typename T>
__global__ void mr2_combine_kernel(const T* yd, const T* yl, const double* coef, T* y, int64_t n, int nz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nz) return;
  const int z = (int)(e / n);
  const double a = coef[2 * z], c = coef[2 * z + 1];
  double v = a * (double)yd[e];
  if (c != 0.0) v += c * (double)yl[e];
  y[e] = (T)v;
}

static unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_bias_act(float* pre, float* post, const float* bias, int n, int w, int act, hipStream_t s) {
  hipLaunchKernelGGL(bias_act_kernel, dim3(nb256((int64_t)n * w)), dim3(256), 0, s, pre, post, bias, n, w, act);
  return hipGetLastError();
}
hipError_t launch_dact(float* g, const float* pre, int64_t total, hipStream_t s) {
  hipLaunchKernelGGL(dact_kernel, dim3(nb256(total)), dim3(256), 0, s, g, pre, total);
  return hipGetLastError();
}
hipError_t launch_colsum(const float* g, int n, int w, float* db, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3(w), dim3(256), 0, s, g, n, w, db);
  return hipGetLastError();
}
// *x = 0 by a kernel (no memset node when the caller captures a graph)
__global__ void zero_double_kernel(double* x) { *x = 0.0; }

hipError_t launch_zero_double(double* x, hipStream_t s) {
  hipLaunchKernelGGL(zero_double_kernel, dim3(1), dim3(1), 0, s, x);
  return hipGetLastError();
}

hipError_t launch_mse(const float* Y, const float* Tg, float* dY, int64_t total, double* loss, hipStream_t s) {
  hipLaunchKernelGGL(mse_kernel, dim3(nb256(total)), dim3(256), 0, s, Y, Tg, dY, total, 1.0 / (double)total, loss);
  return hipGetLastError();
}
hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(nb256(n)), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t launch_features(int ctype, const void* b, const void* d, int64_t n, int nz, double* scales, float* X,
                           hipStream_t s) {
  const int ntiles = (int)((n + 63) / 64);
  if (ctype == 0) {
    hipLaunchKernelGGL(feat_scale_kernel<double>, dim3(nz), dim3(256), 0, s, (const double*)b, (const double*)d, n,
                       scales);
    hipLaunchKernelGGL(feat_kernel<double>, dim3(nb256((int64_t)ntiles * 128 * nz)), dim3(256), 0, s,
                       (const double*)b, (const double*)d, n, ntiles, scales, X, nz);
  } else {
    hipLaunchKernelGGL(feat_scale_kernel<float>, dim3(nz), dim3(256), 0, s, (const float*)b, (const float*)d, n,
                       scales);
    hipLaunchKernelGGL(feat_kernel<float>, dim3(nb256((int64_t)ntiles * 128 * nz)), dim3(256), 0, s,
                       (const float*)b, (const float*)d, n, ntiles, scales, X, nz);
  }
  return hipGetLastError();
}
hipError_t launch_targets(int ctype, const void* y, const void* b, const void* d, int64_t n, int nz,
                          const double* scales, float* Yt, hipStream_t s) {
  const int ntiles = (int)((n + 63) / 64);
  if (ctype == 0)
    hipLaunchKernelGGL(target_kernel<double>, dim3(nb256((int64_t)ntiles * 64 * nz)), dim3(256), 0, s,
                       (const double*)y, (const double*)b, (const double*)d, n, ntiles, scales, Yt, nz);
  else
    hipLaunchKernelGGL(target_kernel<float>, dim3(nb256((int64_t)ntiles * 64 * nz)), dim3(256), 0, s,
                       (const float*)y, (const float*)b, (const float*)d, n, ntiles, scales, Yt, nz);
  return hipGetLastError();
}
hipError_t launch_untile(int ctype, const float* Yn, int64_t n, int nz, const double* scales, void* y, hipStream_t s) {
  const int ntiles = (int)((n + 63) / 64);
  if (ctype == 0)
    hipLaunchKernelGGL(untile_kernel<double>, dim3(nb256(n * nz)), dim3(256), 0, s, Yn, n, ntiles, scales, (double*)y,
                       nz);
  else
    hipLaunchKernelGGL(untile_kernel<float>, dim3(nb256(n * nz)), dim3(256), 0, s, Yn, n, ntiles, scales, (float*)y,
                       nz);
  return hipGetLastError();
}
hipError_t launch_mr2(int ctype, const void* Pd, const void* Pl, const void* b, int64_t n, int nz, double* coef,
                      hipStream_t s) {
  if (ctype == 0)
    hipLaunchKernelGGL(mr2_kernel<double>, dim3(nz), dim3(256), 0, s, (const double*)Pd, (const double*)Pl,
                       (const double*)b, n, coef);
  else
    hipLaunchKernelGGL(mr2_kernel<float>, dim3(nz), dim3(256), 0, s, (const float*)Pd, (const float*)Pl,
                       (const float*)b, n, coef);
  return hipGetLastError();
}
hipError_t launch_mr2_combine(int ctype, const void* yd, const void* yl, const double* coef, void* y, int64_t n,
                              int nz, hipStream_t s) {
  if (ctype == 0)
    hipLaunchKernelGGL(mr2_combine_kernel<double>, dim3(nb256(n * nz)), dim3(256), 0, s, (const double*)yd,
                       (const double*)yl, coef, (double*)y, n, nz);
  else
    hipLaunchKernelGGL(mr2_combine_kernel<float>, dim3(nb256(n * nz)), dim3(256), 0, s, (const float*)yd,
                       (const float*)yl, coef, (float*)y, n, nz);
  return hipGetLastError();
}

}  // namespace ttn
