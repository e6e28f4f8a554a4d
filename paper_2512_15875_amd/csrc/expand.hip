// Bond expansion: the rank-revealing completion of one node's basis
// (Sec. II.C.2 dynamic bond dimensions; used when the maximum bond grows
// between the LOBPCG and inverse-iteration stages, Sec. III.B).
//
// Per state (one workgroup each), with m = rows of the node's local space:
//   A = [Q | S]   Q: the current orthonormal basis (D columns), S: n sketch
//                 columns of the local H x (the parent leg probed);
//   Householder QR of A, the D columns of Q taken first without pivoting, then
//   `grow` steps each bringing forward the remaining column of largest norm
//   below the diagonal (the first one on ties);
//   Y = [Q, q_D, ..., q_{D+grow-1}] with q_c = H_0 H_1 ... H_c e_c signed so
//   that R's diagonal entry c is >= 0.
// The completions are orthogonal to Q by construction, also where the sketch
// has fewer independent directions than the growth.  Columns are contiguous
// runs of m elements (the parent leg is a node tensor's slowest leg); dot
// products and norms are summed in FP64, one wave per column.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "wave.h"

namespace ttn {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void expand_complete_kernel(const T* __restrict__ Qx, int64_t qstride,
                                                              const T* __restrict__ S, int64_t sstride, T* A,
                                                              int64_t astride, T* Y, int64_t ystride, int D, int n,
                                                              int grow, int m) {
  __shared__ double nrm[256], vvs[256], dg[256], red[4];
  __shared__ int piv;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int j = blockIdx.x;
  const T* q = Qx + (int64_t)j * qstride;
  const T* s = S + (int64_t)j * sstride;
  T* a = A + (int64_t)j * astride;
  T* y = Y + (int64_t)j * ystride;
  const int nc = D + n, K = D + grow;
  for (int64_t e = tid; e < (int64_t)D * m; e += 256) a[e] = q[e];
  for (int64_t e = tid; e < (int64_t)n * m; e += 256) a[(int64_t)D * m + e] = s[e];
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    if (k >= D) {
      // pivot: the remaining column of largest norm in rows k..m-1
      for (int c = k + wid; c < nc; c += 4) {
        const T* col = a + (int64_t)c * m;
        double acc = 0.0;
        for (int r = k + lane; r < m; r += 64) acc += (double)col[r] * (double)col[r];
        acc = wave_sum_dpp(acc);
        if (lane == 0) nrm[c] = acc;
      }
      __syncthreads();
      if (tid == 0) {
        int best = k;
        for (int c = k + 1; c < nc; ++c)
          if (nrm[c] > nrm[best]) best = c;
        piv = best;
      }
      __syncthreads();
      const int p = piv;
      if (p != k)
        for (int r = tid; r < m; r += 256) {
          const T t = a[(int64_t)k * m + r];
          a[(int64_t)k * m + r] = a[(int64_t)p * m + r];
          a[(int64_t)p * m + r] = t;
        }
      __syncthreads();
    }
    // reflector from column k, rows k..m-1: v = x + sign(x_0) |x| e_1, stored in place
    T* ck = a + (int64_t)k * m;
    double part = 0.0;
    for (int r = k + tid; r < m; r += 256) part += (double)ck[r] * (double)ck[r];
    part = wave_sum_dpp(part);
    if (lane == 0) red[wid] = part;
    __syncthreads();
    const double nx2 = (red[0] + red[1]) + (red[2] + red[3]);
    const double alpha = (double)ck[k];
    const double sg = alpha >= 0.0 ? 1.0 : -1.0;
    const double nx = sqrt(nx2);
    const double v0 = alpha + sg * nx;
    const double vv = nx2 - alpha * alpha + v0 * v0;
    __syncthreads();  // every thread has read ck[k] before it changes
    if (tid == 0) {
      ck[k] = (T)v0;
      vvs[k] = vv;
      dg[k] = -sg * nx;
    }
    __syncthreads();
    if (vv > 0.0)
      for (int c = k + 1 + wid; c < nc; c += 4) {
        T* col = a + (int64_t)c * m;
        double acc = 0.0;
        for (int r = k + lane; r < m; r += 64) acc += (double)ck[r] * (double)col[r];
        acc = wave_sum_dpp(acc);
        const double f = 2.0 * acc / vv;
        for (int r = k + lane; r < m; r += 64) col[r] = (T)((double)col[r] - f * (double)ck[r]);
      }
    __syncthreads();
  }
  // the basis: Q first, then the completions q_c = H_0 ... H_c e_c
  for (int64_t e = tid; e < (int64_t)D * m; e += 256) y[e] = q[e];
  for (int c = D + wid; c < K; c += 4) {
    T* col = y + (int64_t)c * m;
    for (int r = lane; r < m; r += 64) col[r] = (T)(r == c ? 1.0 : 0.0);
    for (int h = c; h >= 0; --h) {
      const double vvh = vvs[h];
      if (!(vvh > 0.0)) continue;
      const T* vh = a + (int64_t)h * m;
      double acc = 0.0;
      for (int r = h + lane; r < m; r += 64) acc += (double)vh[r] * (double)col[r];
      acc = wave_sum_dpp(acc);
      const double f = 2.0 * acc / vvh;
      for (int r = h + lane; r < m; r += 64) col[r] = (T)((double)col[r] - f * (double)vh[r]);
    }
    if (dg[c] < 0.0)
      for (int r = lane; r < m; r += 64) col[r] = -col[r];
  }
}

}  // namespace

hipError_t launch_expand_complete(int ctype, const void* Qx, int64_t qstride, const void* S, int64_t sstride, void* A,
                                  int64_t astride, void* Y, int64_t ystride, int D, int n, int grow, int m, int k,
                                  hipStream_t s) {
  if (k <= 0) return hipSuccess;
  if (ctype == 0)
    hipLaunchKernelGGL(expand_complete_kernel<double>, dim3((unsigned)k), dim3(256), 0, s, (const double*)Qx, qstride,
                       (const double*)S, sstride, (double*)A, astride, (double*)Y, ystride, D, n, grow, m);
  else
    hipLaunchKernelGGL(expand_complete_kernel<float>, dim3((unsigned)k), dim3(256), 0, s, (const float*)Qx, qstride,
                       (const float*)S, sstride, (float*)A, astride, (float*)Y, ystride, D, n, grow, m);
  return hipGetLastError();
}

}  // namespace ttn
