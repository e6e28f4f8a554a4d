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

}  // namespace ttn
