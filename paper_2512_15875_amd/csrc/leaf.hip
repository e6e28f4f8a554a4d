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

}  // namespace ttn
