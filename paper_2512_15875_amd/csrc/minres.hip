// Batched MINRES for the k local systems (H_eff,j - s_j) y_j = b_j of a sweep
// step (Sec. II.C.3: local solves by MINRES), after Paige and Saunders:
// Lanczos tridiagonalisation with the least-squares problem solved by Givens
// rotations.  One workgroup of 1024 threads owns one state: its dot products
// and norms are workgroup reductions in double (wave sums, then 16 partials),
// its scalar recurrence lives in `st`, and the vector updates of an iteration
// are fused into one pass.  The matrix-vector
// product between iterations is heff_apply_block over all k states.
// Converged states are masked (their workgroups return at once).
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"
#include "wave.h"

namespace ttn {

#define MR_NT 1024  // threads per state (16 wave64s)

// workgroup sum: wave reductions (DPP, wave-uniform), then the 16 wave
// partials (red: >= 16 doubles); every thread of the workgroup takes part
__device__ __forceinline__ double wg_sum(double v, double* red) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  v = wave_sum_dpp(v);
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = 0;
#pragma unroll
  for (int i = 0; i < MR_NT / 64; ++i) r += red[i];
  __syncthreads();
  return r;
}

// r = b - Ax0 -> v = r/beta1 ; zero v_prev, d buffers ; scalars
template <typename T>
__global__ __launch_bounds__(MR_NT) void minres_init(const T* b, const T* Ax, T* v, T* vprev, T* d1, T* d2, int64_t n,
                                                   double rtol, MinresState* st, int32_t* active) {
  __shared__ double red[MR_NT / 64];
  const int z = blockIdx.x, t = threadIdx.x;
  const T* bz = b + (int64_t)z * n;
  const T* az = Ax + (int64_t)z * n;
  T* vz = v + (int64_t)z * n;
  double rr = 0, bb = 0;
  for (int64_t i = t; i < n; i += MR_NT) {
    const double r = (double)bz[i] - (double)az[i];
    rr += r * r;
    bb += (double)bz[i] * (double)bz[i];
  }
  rr = wg_sum(rr, red);
  bb = wg_sum(bb, red);
  const double beta1 = sqrt(rr), tol = rtol * sqrt(bb);
  const bool done = !(beta1 > tol) || beta1 == 0.0;
  for (int64_t i = t; i < n; i += MR_NT) {
    const double r = (double)bz[i] - (double)az[i];
    vz[i] = done ? (T)0 : (T)(r / beta1);
    vprev[(int64_t)z * n + i] = (T)0;
    d1[(int64_t)z * n + i] = (T)0;
    d2[(int64_t)z * n + i] = (T)0;
  }
  if (t == 0) {
    MinresState s;
    s.beta = 0;
    s.c1 = 1;
    s.s1 = 0;
    s.c2 = 1;
    s.s2 = 0;
    s.phibar = beta1;
    s.tol = tol;
    s.done = done ? 1 : 0;
    s.iters = 0;
    st[z] = s;
    if (z == 0 && active) *active = (int32_t)gridDim.x;  // the gate opens; minres_count refines it
  }
}

// one MINRES step for every active state.  p holds A v on entry.
// d_new is written into dpp (whose old contents, d_{k-2}, are consumed first);
// v_new = p / beta_next is written into vprev (old v_{k-1} consumed first).
template <typename T>
__global__ __launch_bounds__(MR_NT) void minres_step(T* x, T* v, T* vprev, T* p, const T* dp, T* dpp, int64_t n,
                                                   MinresState* st) {
  __shared__ double red[MR_NT / 64];
  __shared__ MinresState s;
  __shared__ double sh[6];  // eps, delta, gamma, tau, beta_next, alive
  const int z = blockIdx.x, t = threadIdx.x;
  if (t == 0) s = st[z];
  __syncthreads();
  if (s.done) return;
  T* xz = x + (int64_t)z * n;
  T* vz = v + (int64_t)z * n;
  T* vpz = vprev + (int64_t)z * n;
  T* pz = p + (int64_t)z * n;
  const T* dz = dp + (int64_t)z * n;
  T* dppz = dpp + (int64_t)z * n;
  double a = 0;
  for (int64_t i = t; i < n; i += MR_NT) a += (double)vz[i] * (double)pz[i];
  const double alpha = wg_sum(a, red);
  double nn = 0;
  for (int64_t i = t; i < n; i += MR_NT) {
    const double q = (double)pz[i] - alpha * (double)vz[i] - s.beta * (double)vpz[i];
    pz[i] = (T)q;
    nn += q * q;
  }
  const double bn = sqrt(wg_sum(nn, red));
  if (t == 0) {
    const double eps = s.s1 * s.beta;
    const double dbar = s.c1 * s.beta;
    const double delta = s.c2 * dbar + s.s2 * alpha;
    const double gbar = -s.s2 * dbar + s.c2 * alpha;
    const double gamma = hypot(gbar, bn);
    sh[0] = eps;
    sh[1] = delta;
    sh[2] = gamma;
    sh[4] = bn;
    if (gamma == 0.0) {
      s.done = 1;
      sh[5] = 0;
    } else {
      const double c = gbar / gamma, sn = bn / gamma;
      sh[3] = c * s.phibar;
      s.phibar = -sn * s.phibar;
      s.c1 = s.c2;
      s.s1 = s.s2;
      s.c2 = c;
      s.s2 = sn;
      s.iters += 1;
      s.beta = bn;
      if (fabs(s.phibar) <= s.tol || bn == 0.0) s.done = 1;
      sh[5] = 1;
    }
  }
  __syncthreads();
  if (sh[5] != 0) {
    const double eps = sh[0], delta = sh[1], gamma = sh[2], tau = sh[3], bnext = sh[4];
    for (int64_t i = t; i < n; i += MR_NT) {
      const double dn = ((double)vz[i] - delta * (double)dz[i] - eps * (double)dppz[i]) / gamma;
      dppz[i] = (T)dn;
      xz[i] = (T)((double)xz[i] + tau * dn);
      vpz[i] = (T)(bnext > 0 ? (double)pz[i] / bnext : 0.0);
    }
  }
  if (t == 0) st[z] = s;
}


template <typename T>
__global__ void minres_report(const MinresState* st, int k, int32_t* iters, double* resid, int32_t* n_active) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= k) return;
  if (iters) iters[z] = st[z].iters;
  if (resid) resid[z] = fabs(st[z].phibar);
  if (n_active && !st[z].done) atomicAdd(n_active, 1);
}

hipError_t launch_minres_init(int ctype, const void* b, const void* Ax, void* v, void* vprev, void* d1, void* d2,
                              int64_t n, int k, double rtol, MinresState* st, int32_t* active, hipStream_t s) {
  if (ctype == 0)
    hipLaunchKernelGGL(minres_init<double>, dim3(k), dim3(MR_NT), 0, s, (const double*)b, (const double*)Ax, (double*)v,
                       (double*)vprev, (double*)d1, (double*)d2, n, rtol, st, active);
  else
    hipLaunchKernelGGL(minres_init<float>, dim3(k), dim3(MR_NT), 0, s, (const float*)b, (const float*)Ax, (float*)v,
                       (float*)vprev, (float*)d1, (float*)d2, n, rtol, st, active);
  return hipGetLastError();
}

// *active = number of states whose MINRES has not converged (one workgroup;
// written, not accumulated, so no clearing is needed before it)
__global__ __launch_bounds__(256) void minres_count_kernel(const MinresState* st, int k, int32_t* active) {
  __shared__ int part[4];
  int c = 0;
  for (int z = threadIdx.x; z < k; z += 256) c += st[z].done ? 0 : 1;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) *active = part[0] + part[1] + part[2] + part[3];
}

hipError_t launch_minres_count(const MinresState* st, int k, int32_t* active, hipStream_t s) {
  hipLaunchKernelGGL(minres_count_kernel, dim3(1), dim3(256), 0, s, st, k, active);
  return hipGetLastError();
}

hipError_t launch_minres_step(int ctype, void* x, void* v, void* vprev, void* p, const void* dp, void* dpp, int64_t n,
                              int k, MinresState* st, hipStream_t s) {
  if (ctype == 0)
    hipLaunchKernelGGL(minres_step<double>, dim3(k), dim3(MR_NT), 0, s, (double*)x, (double*)v, (double*)vprev,
                       (double*)p, (const double*)dp, (double*)dpp, n, st);
  else
    hipLaunchKernelGGL(minres_step<float>, dim3(k), dim3(MR_NT), 0, s, (float*)x, (float*)v, (float*)vprev, (float*)p,
                       (const float*)dp, (float*)dpp, n, st);
  return hipGetLastError();
}

hipError_t launch_minres_report(const MinresState* st, int k, int32_t* iters, double* resid, int32_t* n_active,
                                hipStream_t s) {
  hipLaunchKernelGGL(minres_report<double>, dim3((k + 255) / 256), dim3(256), 0, s, st, k, iters, resid, n_active);
  return hipGetLastError();
}

// y = b / diag  (the DIAG local map), elementwise with a guard for |diag| tiny
template <typename T>
__global__ void diag_solve_kernel(const T* b, const T* dg, T* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = (double)dg[i];
  y[i] = (T)(fabs(d) > 1e-300 ? (double)b[i] / d : 0.0);
}

hipError_t launch_diag_solve(int ctype, const void* b, const void* dg, void* y, int64_t n, hipStream_t s) {
  const unsigned g = (unsigned)((n + 255) / 256);
  if (ctype == 0)
    hipLaunchKernelGGL(diag_solve_kernel<double>, dim3(g), dim3(256), 0, s, (const double*)b, (const double*)dg,
                       (double*)y, n);
  else
    hipLaunchKernelGGL(diag_solve_kernel<float>, dim3(g), dim3(256), 0, s, (const float*)b, (const float*)dg, (float*)y,
                       n);
  return hipGetLastError();
}

// coef_perm[i] = coef[perm[i]]
__global__ void gather_coef_kernel(const double* coef, const int32_t* perm, int n, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = coef[perm[i]];
}

hipError_t launch_gather_coef(const double* coef, const int32_t* perm, int n, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_coef_kernel, dim3((n + 255) / 256), dim3(256), 0, s, coef, perm, n, out);
  return hipGetLastError();
}

}  // namespace ttn

namespace ttn {

// y[t][i] = sum_{j in seg(t)} coef[j] * S[j][i]  (CSR over targets; rows of
// S are per-term local results); one workgroup row-chunk per target
template <typename T>
__global__ void seg_sum_kernel(const T* S, const int32_t* ptr, const int32_t* terms, const double* coef, T* y,
                               int64_t n, int k) {
  const int t = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k || i >= n) return;
  double acc = 0.0;
  int q = ptr[t];
  const int qe = ptr[t + 1];
  // eight terms' loads in flight, summed in term order (same result as one at
  // a time); the next eight term indices are read while this batch's
  // coefficients and rows are in flight
  int jn[8];
  if (q + 8 <= qe) {
#pragma unroll
    for (int u = 0; u < 8; ++u) jn[u] = terms[q + u];
  }
  for (; q + 8 <= qe; q += 8) {
    int jj[8];
    double cc[8], sv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) jj[u] = jn[u];
    if (q + 16 <= qe) {
#pragma unroll
      for (int u = 0; u < 8; ++u) jn[u] = terms[q + 8 + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      cc[u] = coef[jj[u]];
      sv[u] = (double)S[(int64_t)jj[u] * n + i];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += cc[u] * sv[u];
  }
  for (; q < qe; ++q) {
    const int j = terms[q];
    acc += coef[j] * (double)S[(int64_t)j * n + i];
  }
  y[(int64_t)t * n + i] = (T)acc;
}

hipError_t launch_seg_sum(int ctype, const void* S, const int32_t* ptr, const int32_t* terms, const double* coef,
                          void* y, int64_t n, int k, bool accumulate_first, hipStream_t s) {
  (void)accumulate_first;
  dim3 g((unsigned)((n + 255) / 256), (unsigned)k);
  if (ctype == 0)
    hipLaunchKernelGGL(seg_sum_kernel<double>, g, dim3(256), 0, s, (const double*)S, ptr, terms, coef, (double*)y, n, k);
  else
    hipLaunchKernelGGL(seg_sum_kernel<float>, g, dim3(256), 0, s, (const float*)S, ptr, terms, coef, (float*)y, n, k);
  return hipGetLastError();
}

}  // namespace ttn

namespace ttn {
template <typename T>
__global__ void add_kernel(const T* x, T* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (T)((double)y[i] + (double)x[i]);
}
// r = b - p (the FP64 residual of a refinement step); z = 0
template <typename T>
__global__ void resid_zero_kernel(const T* b, const T* p, T* r, T* zero, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    r[i] = (T)((double)b[i] - (double)p[i]);
    zero[i] = (T)0;
  }
}
hipError_t launch_resid_zero(int ctype, const void* b, const void* p, void* r, void* zero, int64_t n, hipStream_t s) {
  const unsigned g = (unsigned)((n + 255) / 256);
  if (ctype == 0)
    hipLaunchKernelGGL(resid_zero_kernel<double>, dim3(g), dim3(256), 0, s, (const double*)b, (const double*)p,
                       (double*)r, (double*)zero, n);
  else
    hipLaunchKernelGGL(resid_zero_kernel<float>, dim3(g), dim3(256), 0, s, (const float*)b, (const float*)p, (float*)r,
                       (float*)zero, n);
  return hipGetLastError();
}

hipError_t launch_axpy_rows(int ctype, const void* x, void* y, int64_t n, hipStream_t s) {
  const unsigned g = (unsigned)((n + 255) / 256);
  if (ctype == 0) hipLaunchKernelGGL(add_kernel<double>, dim3(g), dim3(256), 0, s, (const double*)x, (double*)y, n);
  else hipLaunchKernelGGL(add_kernel<float>, dim3(g), dim3(256), 0, s, (const float*)x, (float*)y, n);
  return hipGetLastError();
}
}  // namespace ttn
