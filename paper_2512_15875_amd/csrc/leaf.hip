// Fused H_eff product at a node with one virtual leg and a physical leg (the
// leaves of a tree, the ends of an MPS), Sec. II.C.3: for one state
//   Y[b][p] = alpha (sum_{w, a, q} E[b][w][a] W[w][p][q] X[a][q] - s X[b][p]) (+ Y)
// with E the environment of the single neighbour (bra bond b, operator bond w,
// ket bond a) and W the node's operator tensor (operator bond, output, input).
// The staged path runs this as two small contractions through an HBM
// intermediate, two launches per product; here one workgroup per state stages
// X, E and W in LDS, forms T[b][w][q] = sum_a E[b][w][a] X[a][q] there and
// finishes with the W contraction and the epilogue.  The work per state is a
// few thousand flops, so it runs on the vector ALUs.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "wave.h"

namespace ttn {

template <typename T>
__global__ __launch_bounds__(256) void leaf_heff_kernel(LeafHeffArgs g) {
  extern __shared__ unsigned char leaf_smem[];
  T* sX = reinterpret_cast<T*>(leaf_smem);
  const int Db = g.Db, M = g.M, Da = g.Da, d = g.d;
  T* sE = sX + Da * d;        // [Db][M][Da]
  T* sW = sE + Db * M * Da;   // [M][d][d]
  T* sT = sW + M * d * d;     // [Db][M][d]
  const int z = blockIdx.x, tid = threadIdx.x;
  if (z >= g.n || (g.gate && *g.gate == 0)) return;  // uniform per workgroup, before any barrier
  int xr = g.x_ids ? g.x_ids[z] : z;
  int er = g.pair_ids ? g.pair_ids[z] : z;
  int yr = g.y_ids ? g.y_ids[z] : z;
  if (xr < 0 || xr >= g.x_rows || er < 0 || er >= g.n_slots || yr < 0 || yr >= g.y_rows) {  // clamp and report
    if (tid == 0) atomicOr(g.flag + 2, 1);
    xr = xr < 0 ? 0 : (xr >= g.x_rows ? g.x_rows - 1 : xr);
    er = er < 0 ? 0 : (er >= g.n_slots ? g.n_slots - 1 : er);
    yr = yr < 0 ? 0 : (yr >= g.y_rows ? g.y_rows - 1 : yr);
  }
  const T* __restrict__ X = (const T*)g.X + (int64_t)xr * g.x_stride;
  const T* __restrict__ E = (const T*)g.E + (int64_t)er * g.e_stride;
  const T* __restrict__ W = (const T*)g.W;
  T* __restrict__ Y = (T*)g.Y + (int64_t)yr * g.y_stride;
  for (int i = tid; i < Da * d; i += 256) sX[i] = X[i];
  for (int i = tid; i < Db * M * Da; i += 256) sE[i] = E[i];
  for (int i = tid; i < M * d * d; i += 256) sW[i] = W[i];
  __syncthreads();
  // T[b][w][q] = sum_a E[b][w][a] X[a][q]
  for (int e = tid; e < Db * M * d; e += 256) {
    const int bw = e / d, q = e - bw * d;
    const T* er_ = sE + bw * Da;
    T acc = 0;
    for (int a = 0; a < Da; ++a) acc += er_[a] * sX[a * d + q];
    sT[e] = acc;
  }
  __syncthreads();
  // Y[b][p] = sum_{w, q} T[b][w][q] W[w][p][q], then the epilogue
  const double alpha = g.alpha ? g.alpha[z] : 1.0;
  const double sh = g.shift ? g.shift[z] : 0.0;
  for (int e = tid; e < Db * d; e += 256) {
    const int b = e / d, p = e - b * d;
    T acc = 0;
    for (int w = 0; w < M; ++w) {
      const T* tr = sT + (b * M + w) * d;
      const T* wr = sW + (w * d + p) * d;
      for (int q = 0; q < d; ++q) acc += tr[q] * wr[q];
    }
    double v = (double)acc;
    if (g.shift) v -= sh * (double)sX[e];  // square bonds: X[b][p] sits at the same flat index
    v *= alpha;
    if (g.accum) v += (double)Y[e];
    Y[e] = (T)v;
  }
}

size_t leaf_heff_lds_bytes(int Db, int M, int Da, int d, int esize) {
  return (size_t)esize * ((size_t)Da * d + (size_t)Db * M * Da + (size_t)M * d * d + (size_t)Db * M * d);
}

hipError_t launch_leaf_heff(int ctype, const LeafHeffArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const size_t bytes = leaf_heff_lds_bytes(a.Db, a.M, a.Da, a.d, ctype == 0 ? 8 : 4);
  if (ctype == 0)
    hipLaunchKernelGGL(leaf_heff_kernel<double>, dim3(a.n), dim3(256), bytes, s, a);
  else
    hipLaunchKernelGGL(leaf_heff_kernel<float>, dim3(a.n), dim3(256), bytes, s, a);
  return hipGetLastError();
}

// The ALS local solve (H_eff - s) y = b at a leaf (Sec. II.C.3) in one launch:
// one workgroup per state runs the warm-start product, the initialisation and
// every MINRES iteration of the batched kernels (the same Paige-Saunders
// recurrence and the same storage roundings: vectors stored in T, products and
// updates in double), with E and W staged in LDS once, a thread per vector
// element holding x, v, v_prev, d, d_prev in registers, and the product of the
// leaf kernel above between the steps.  A state stops at convergence or after
// maxiter iterations, as its batched solve does.  The staged form issues two
// launches per iteration for every leaf solve.
template <typename T>
__global__ __launch_bounds__(256) void leaf_minres_kernel(LeafHeffArgs g, const T* bvec, T* y, int64_t n, double rtol,
                                                          int maxiter, MinresState* st) {
  extern __shared__ unsigned char lm_smem[];
  const int Db = g.Db, M = g.M, Da = g.Da, d = g.d;
  T* sX = reinterpret_cast<T*>(lm_smem);  // [Da][d]
  T* sE = sX + Da * d;                     // [Db][M][Da]
  T* sW = sE + Db * M * Da;                // [M][d][d]
  T* sT = sW + M * d * d;                  // [Db][M][d]
  __shared__ double red[4];
  const int z = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const T* __restrict__ E = (const T*)g.E + (int64_t)z * g.e_stride;
  const T* __restrict__ W = (const T*)g.W;
  for (int i = t; i < Db * M * Da; i += 256) sE[i] = E[i];
  for (int i = t; i < M * d * d; i += 256) sW[i] = W[i];
  const double sh = g.shift ? g.shift[z] : 0.0;
  const bool own = t < n;
  T* yz = y + (int64_t)z * n;
  T xv = own ? yz[t] : T(0);
  const T bv = own ? bvec[(int64_t)z * n + t] : T(0);
  // (H_eff - s) applied to the vector whose element t this thread holds, as
  // the leaf kernel computes it; every thread takes part (barriers)
  auto apply = [&](T in) -> T {
    __syncthreads();  // earlier readers of sX and sT are done (and E, W staged)
    if (own) sX[t] = in;
    __syncthreads();
    for (int e = t; e < Db * M * d; e += 256) {
      const int bw = e / d, q = e - bw * d;
      const T* er = sE + bw * Da;
      T acc = 0;
      for (int a = 0; a < Da; ++a) acc += er[a] * sX[a * d + q];
      sT[e] = acc;
    }
    __syncthreads();
    if (!own) return T(0);
    const int b = t / d, p = t - b * d;
    T acc = 0;
    for (int w = 0; w < M; ++w) {
      const T* tr = sT + (b * M + w) * d;
      const T* wr = sW + (w * d + p) * d;
      for (int q = 0; q < d; ++q) acc += tr[q] * wr[q];
    }
    double v = (double)acc;
    if (g.shift) v -= sh * (double)sX[t];
    return (T)v;
  };
  auto bsum = [&](double v) -> double {
    v = wave_sum_dpp(v);
    if (lane == 0) red[wv] = v;
    __syncthreads();
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
  };
  // initialisation from the warm start: r = b - A x, v = r / |r|
  const T ax = apply(xv);
  const double r0 = own ? (double)bv - (double)ax : 0.0;
  const double rr = bsum(r0 * r0);
  const double bb = bsum(own ? (double)bv * (double)bv : 0.0);
  const double beta1 = sqrt(rr), tol = rtol * sqrt(bb);
  bool done = !(beta1 > tol) || beta1 == 0.0;
  T v = (own && !done) ? (T)(r0 / beta1) : T(0);
  T vp = 0, dp = 0, dpp = 0;
  double beta = 0, c1 = 1, s1 = 0, c2 = 1, s2 = 0, phibar = beta1;
  int iters = 0;
  for (int it = 0; it < maxiter && !done; ++it) {  // uniform: every thread holds the same scalars
    const T pv = apply(v);
    const double alpha = bsum(own ? (double)v * (double)pv : 0.0);
    const double q = own ? (double)pv - alpha * (double)v - beta * (double)vp : 0.0;
    const T qT = (T)q;
    const double bn = sqrt(bsum(q * q));
    const double eps = s1 * beta, dbar = c1 * beta;
    const double delta = c2 * dbar + s2 * alpha;
    const double gbar = -s2 * dbar + c2 * alpha;
    const double gamma = hypot(gbar, bn);
    if (gamma == 0.0) {
      done = true;
      break;
    }
    const double c = gbar / gamma, sn = bn / gamma;
    const double tau = c * phibar;
    phibar = -sn * phibar;
    c1 = c2;
    s1 = s2;
    c2 = c;
    s2 = sn;
    iters += 1;
    beta = bn;
    if (fabs(phibar) <= tol || bn == 0.0) done = true;
    const double dn = ((double)v - delta * (double)dp - eps * (double)dpp) / gamma;
    xv = (T)((double)xv + tau * dn);
    const T vn = (T)(bn > 0 ? (double)qT / bn : 0.0);
    vp = v;
    v = vn;
    dpp = dp;
    dp = (T)dn;
  }
  if (own) yz[t] = xv;
  if (t == 0) {
    MinresState s;
    s.beta = beta;
    s.c1 = c1;
    s.s1 = s1;
    s.c2 = c2;
    s.s2 = s2;
    s.phibar = phibar;
    s.tol = tol;
    s.done = done ? 1 : 0;
    s.iters = iters;
    st[z] = s;
  }
}

hipError_t launch_leaf_minres(int ctype, const LeafHeffArgs& a, const void* b, void* y, int64_t n, double rtol,
                              int maxiter, MinresState* st, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (n > 256 || n != (int64_t)a.Da * a.d || a.Da != a.Db) return hipErrorInvalidValue;
  const size_t bytes = leaf_heff_lds_bytes(a.Db, a.M, a.Da, a.d, ctype == 0 ? 8 : 4);
  if (ctype == 0)
    hipLaunchKernelGGL(leaf_minres_kernel<double>, dim3(a.n), dim3(256), bytes, s, a, (const double*)b, (double*)y, n,
                       rtol, maxiter, st);
  else
    hipLaunchKernelGGL(leaf_minres_kernel<float>, dim3(a.n), dim3(256), bytes, s, a, (const float*)b, (float*)y, n,
                       rtol, maxiter, st);
  return hipGetLastError();
}

}  // namespace ttn
