// Small memory-bound kernels of the hot path: diagonal gathers for diag(H_eff),
// and the vector helpers of the eigensolver drivers (square roots of squared
// norms, coefficient gathers, dtype conversion of state blocks).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ttn {

// Wd[w..., p] = W[w..., p, p]
template <typename T>
__global__ void wdiag_kernel(const T* W, int64_t nw, int d, T* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nw * d) return;
  const int64_t w = i / d;
  const int p = (int)(i - w * d);
  out[i] = W[(w * d + p) * d + p];
}

// Ed[z][b][w] = E[pair(z)][b][w][b]
template <typename T>
__global__ void ediag_kernel(const T* E, const int32_t* pair, int n_slots, int* flag, int64_t estride, int B, int Mw,
                             int nz, T* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)B * Mw;
  if (i >= per * nz) return;
  const int z = (int)(i / per);
  const int64_t r = i - (int64_t)z * per;
  const int b = (int)(r / Mw);
  const int w = (int)(r - (int64_t)b * Mw);
  int64_t slot = pair ? pair[z] : z;
  if (slot < 0 || slot >= n_slots) {  // clamp and report instead of reading out of bounds
    atomicOr(flag + 2, 1);
    slot = slot < 0 ? 0 : n_slots - 1;
  }
  out[i] = E[slot * estride + ((int64_t)b * Mw + w) * B + b];
}

template <typename T>
static hipError_t gather_t(const DiagDesc& dd, void* ws, const int64_t* ed_off, int nz, hipStream_t s) {
  int64_t nw = 1;
  for (int i = 0; i < dd.kappa; ++i) nw *= dd.dM[i];
  const int64_t nwd = nw * dd.d;
  hipLaunchKernelGGL(wdiag_kernel<T>, dim3((unsigned)((nwd + 255) / 256)), dim3(256), 0, s, (const T*)dd.W, nw, dd.d,
                     (T*)ws);
  for (int i = 0; i < dd.kappa; ++i) {
    const int64_t n = (int64_t)dd.dB[i] * dd.dM[i] * nz;
    hipLaunchKernelGGL(ediag_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const T*)dd.E[i], dd.pair,
                       dd.n_slots, dd.flag, dd.Estride[i], dd.dB[i], dd.dM[i], nz, (T*)ws + ed_off[i]);
  }
  return hipGetLastError();
}

hipError_t launch_diag_gather(int ctype, const DiagDesc& dd, void* ws, const int64_t* ed_off, int nz, hipStream_t s) {
  if (ctype == 0) return gather_t<double>(dd, ws, ed_off, nz, s);
  return gather_t<float>(dd, ws, ed_off, nz, s);
}

// y[i] = sqrt(x[i])
__global__ void vsqrt_kernel(const double* x, double* y, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = sqrt(x[i]);
}

// dst[i] = idx[i] >= 0 ? src[idx[i]] : fill   (idx < src_n checked on the host side of the table's producer)
__global__ void vgather_kernel(const int32_t* idx, const double* src, int src_n, double fill, double* dst, int n,
                               int* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = idx[i];
  if (j >= src_n) {  // report instead of reading out of bounds
    atomicOr(flag + 2, 1);
    dst[i] = fill;
    return;
  }
  dst[i] = j >= 0 ? src[j] : fill;
}

template <typename S, typename D>
__global__ void convert_kernel(const S* x, D* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (D)x[i];
}

hipError_t launch_vsqrt(const double* x, double* y, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(vsqrt_kernel, dim3((n + 255) / 256), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t launch_vgather(const int32_t* idx, const double* src, int src_n, double fill, double* dst, int n, int* flag,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(vgather_kernel, dim3((n + 255) / 256), dim3(256), 0, s, idx, src, src_n, fill, dst, n, flag);
  return hipGetLastError();
}

// X[z][i][j] = (i == j) for z < k, i, j < n
template <typename T>
__global__ void set_identity_kernel(T* X, int n, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int64_t r = e % ((int64_t)n * n);
  X[e] = (T)((r / n) == (r % n) ? 1.0 : 0.0);
}

hipError_t launch_set_identity(int ctype, void* X, int n, int k, hipStream_t s) {
  const int64_t total = (int64_t)k * n * n;
  if (total <= 0) return hipSuccess;
  const dim3 g((unsigned)((total + 255) / 256));
  if (ctype == 0) hipLaunchKernelGGL(set_identity_kernel<double>, g, dim3(256), 0, s, (double*)X, n, total);
  else hipLaunchKernelGGL(set_identity_kernel<float>, g, dim3(256), 0, s, (float*)X, n, total);
  return hipGetLastError();
}

// sdt / ddt: 0 double, 1 float
hipError_t launch_convert(int sdt, const void* x, int ddt, void* y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 g((unsigned)((n + 255) / 256));
  if (sdt == 1 && ddt == 0) hipLaunchKernelGGL((convert_kernel<float, double>), g, dim3(256), 0, s, (const float*)x, (double*)y, n);
  else if (sdt == 0 && ddt == 1) hipLaunchKernelGGL((convert_kernel<double, float>), g, dim3(256), 0, s, (const double*)x, (float*)y, n);
  else if (sdt == 0) hipLaunchKernelGGL((convert_kernel<double, double>), g, dim3(256), 0, s, (const double*)x, (double*)y, n);
  else hipLaunchKernelGGL((convert_kernel<float, float>), g, dim3(256), 0, s, (const float*)x, (float*)y, n);
  return hipGetLastError();
}


// ---- split Jacobi preconditioning of the local MINRES (one workgroup per
// state for the scale, element-wise products gated like the contraction
// kernels so that a converged batch stops without the host)
namespace {
template <typename T>
__global__ __launch_bounds__(256) void precond_scale_kernel(const T* d, T* dsq, int64_t n, int mode, double damp) {
  __shared__ double red[4];
  const int z = blockIdx.x, t = threadIdx.x;
  const T* dz = d + (int64_t)z * n;
  T* oz = dsq + (int64_t)z * n;
  double g2 = 0.0;
  if (mode == 2) {
    double s = 0.0;
    for (int64_t i = t; i < n; i += 256) s += (double)dz[i] * (double)dz[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((t & 63) == 0) red[t >> 6] = s;
    __syncthreads();
    const double ms = (red[0] + red[1] + red[2] + red[3]) / (double)n;
    g2 = damp * damp * ms;
  }
  for (int64_t i = t; i < n; i += 256) {
    const double v = (double)dz[i] * (double)dz[i] + g2;
    oz[i] = (T)(v > 0.0 ? pow(v, -0.25) : 1.0);
  }
}

template <typename T>
__global__ void ew_mul_kernel(const T* a, const T* b, T* out, int64_t n, const int32_t* gate) {
  if (gate && *gate == 0) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}

template <typename T>
__global__ void ew_div_kernel(const T* a, const T* b, T* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = a[i] / b[i];
}
}  // namespace

hipError_t launch_precond_scale(int ctype, const void* d, void* dsq, int64_t n, int k, int mode, double damp,
                                hipStream_t s) {
  if (k <= 0 || n <= 0) return hipSuccess;
  if (ctype == 0)
    hipLaunchKernelGGL(precond_scale_kernel<double>, dim3((unsigned)k), dim3(256), 0, s, (const double*)d,
                       (double*)dsq, n, mode, damp);
  else
    hipLaunchKernelGGL(precond_scale_kernel<float>, dim3((unsigned)k), dim3(256), 0, s, (const float*)d, (float*)dsq,
                       n, mode, damp);
  return hipGetLastError();
}

hipError_t launch_ew_mul(int ctype, const void* a, const void* b, void* out, int64_t n, const int32_t* gate,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 g((unsigned)((n + 255) / 256));
  if (ctype == 0)
    hipLaunchKernelGGL(ew_mul_kernel<double>, g, dim3(256), 0, s, (const double*)a, (const double*)b, (double*)out, n,
                       gate);
  else
    hipLaunchKernelGGL(ew_mul_kernel<float>, g, dim3(256), 0, s, (const float*)a, (const float*)b, (float*)out, n,
                       gate);
  return hipGetLastError();
}

hipError_t launch_ew_div(int ctype, const void* a, const void* b, void* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 g((unsigned)((n + 255) / 256));
  if (ctype == 0)
    hipLaunchKernelGGL(ew_div_kernel<double>, g, dim3(256), 0, s, (const double*)a, (const double*)b, (double*)out, n);
  else
    hipLaunchKernelGGL(ew_div_kernel<float>, g, dim3(256), 0, s, (const float*)a, (const float*)b, (float*)out, n);
  return hipGetLastError();
}

}  // namespace ttn
