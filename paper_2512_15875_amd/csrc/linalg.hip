// FP64 dense linear algebra of the hot path, on the device:
//  * Rayleigh-Ritz for the LOBPCG / inverse-iteration subspaces (one
//    workgroup per problem): Cholesky of the overlap (SVQB fallback through a
//    eigendecomposition of the overlap), reduction to a standard symmetric
//    problem, tridiagonalisation + implicit QL eigensolver, back-transform;
//  * the QR gauge move of a block (one workgroup per state, Householder);
//  * per-state norms and scaling of node tensors.
// Everything accumulates in double, whatever the storage dtype.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include <cmath>

#include "internal.h"
#include "wave.h"

namespace ttn {

#define NT 1024  // threads per workgroup of the dense kernels

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}


__device__ __forceinline__ double wave_sum64(double v) { return wave_sum_dpp(v); }

#define QL_CH 16  // loads of a row of Z in flight together during the QL rotations

// Symmetric eigendecomposition of the n x n matrix A (row-major, leading dim
// ld, global memory; destroyed).  Householder reduction to tridiagonal form
// A = Q T Q^T with Q formed explicitly in Z (backward accumulation), then the
// implicit QL iteration with a Wilkinson-type shift on T (the classical
// tql2-type scheme, Bowdler, Martin, Reinsch and Wilkinson 1968): one thread
// chases each bulge and records the sweep's plane rotations, then every
// thread applies them to its own rows of Z.  On return the eigenvalues are
// on the diagonal of A and the eigenvectors are the columns of Z.  A QL
// iteration that has not converged after 30 sweeps for one eigenvalue raises
// flag[3].  Shared arrays of at least n doubles: rc, rs, v, w, d, e, tv.
// Inlined into its caller so that the compiler sees which pointers are LDS
// and which global memory (as a called function every access went through
// flat loads and stores that could not be reordered: 20 -> 18 ms at n = 150).
__device__ __forceinline__ void sym_eig(double* A, double* Z, int n, int ld, double* rc, double* rs, double* v, double* w,
                        double* d, double* e, double* tv, double* red, int* flag) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
  __shared__ int s_lo, s_hi;
  // ---- tridiagonalisation: step k zeroes column k below the subdiagonal
  for (int k = 0; k + 2 < n; ++k) {
    const int len = n - k - 1;  // x = A[k+1 .. n-1][k]
    double s2 = 0;
    for (int i = t; i < len; i += blockDim.x) {
      const double x = A[(size_t)(k + 1 + i) * ld + k];
      s2 += x * x;
    }
    s2 = block_sum(s2, red);
    const double x0 = A[(size_t)(k + 1) * ld + k];
    const double nrm = sqrt(s2);
    const double alpha = nrm == 0.0 ? 0.0 : (x0 >= 0 ? -nrm : nrm);
    const double v0 = x0 - alpha;
    const double vn2 = s2 - x0 * x0 + v0 * v0;
    const double tk = vn2 > 0 ? 2.0 / vn2 : 0.0;  // reflector I - tk v v^T, v = x - alpha e_1
    for (int i = t; i < len; i += blockDim.x) v[i] = i == 0 ? v0 : A[(size_t)(k + 1 + i) * ld + k];
    if (t == 0) {
      d[k] = A[(size_t)k * ld + k];
      e[k] = tk == 0.0 ? x0 : alpha;
      tv[k] = tk;
    }
    __syncthreads();
    if (tk == 0.0) continue;  // uniform: nothing to reflect
    // w = tk * A_sub v (one wave per row, lanes along the row)
    for (int i = wv; i < len; i += nw) {
      const double* row = A + (size_t)(k + 1 + i) * ld + (k + 1);
      double sacc = 0;
      for (int j = lane; j < len; j += 64) sacc += row[j] * v[j];
      sacc = wave_sum64(sacc);
      if (lane == 0) w[i] = tk * sacc;
    }
    __syncthreads();
    double pv = 0;
    for (int i = t; i < len; i += blockDim.x) pv += w[i] * v[i];
    pv = block_sum(pv, red);
    const double kc = 0.5 * tk * pv;
    for (int i = t; i < len; i += blockDim.x) w[i] -= kc * v[i];
    __syncthreads();
    // A_sub -= v w^T + w v^T; v kept in column k for Q
    for (int q = t; q < len * len; q += blockDim.x) {
      const int i = q / len, j = q - i * len;
      A[(size_t)(k + 1 + i) * ld + (k + 1 + j)] -= v[i] * w[j] + w[i] * v[j];
    }
    for (int i = t; i < len; i += blockDim.x) A[(size_t)(k + 1 + i) * ld + k] = v[i];
    __syncthreads();
  }
  if (t == 0) {
    if (n >= 2) {
      d[n - 2] = A[(size_t)(n - 2) * ld + (n - 2)];
      e[n - 2] = A[(size_t)(n - 1) * ld + (n - 2)];
    }
    d[n - 1] = A[(size_t)(n - 1) * ld + (n - 1)];
    if (n >= 2) tv[n - 2] = 0.0;
  }
  // ---- Q = H_0 H_1 ... H_{n-3}, accumulated backward into Z
  for (int q = t; q < n * n; q += blockDim.x) {
    const int r = q / n, c = q - r * n;
    Z[(size_t)r * ld + c] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const double tk = tv[k];
    if (tk == 0.0) continue;  // uniform
    const int len = n - k - 1;
    for (int i = t; i < len; i += blockDim.x) v[i] = A[(size_t)(k + 1 + i) * ld + k];
    __syncthreads();
    // w_j = sum_i v_i Z[k+1+i][k+1+j]  (thread per column: coalesced along rows of Z)
    for (int j = t; j < len; j += blockDim.x) {
      double sacc = 0;
#pragma unroll 8
      for (int i = 0; i < len; ++i) sacc += v[i] * Z[(size_t)(k + 1 + i) * ld + (k + 1 + j)];
      w[j] = tk * sacc;
    }
    __syncthreads();
    for (int q = t; q < len * len; q += blockDim.x) {
      const int i = q / len, j = q - i * len;
      Z[(size_t)(k + 1 + i) * ld + (k + 1 + j)] -= v[i] * w[j];
    }
    __syncthreads();
  }
  // ---- implicit QL on (d, e), rotations accumulated into the columns of Z.
  // A subdiagonal entry is negligible below eps times the larger of its two
  // diagonal neighbours and the norm of T (the norm-wise test keeps zero or
  // tiny eigenvalue clusters from stalling the relative one).
  __shared__ double s_tn;
  if (t == 0) {
    double tn = 0;
    for (int i = 0; i < n; ++i) tn = fmax(tn, fabs(d[i]) + (i + 1 < n ? fabs(e[i]) : 0.0));
    s_tn = tn;
  }
  __syncthreads();
  const double tnorm = s_tn;
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      if (t == 0) {
        int m = l;
        for (; m + 1 < n; ++m) {
          const double dd = fabs(d[m]) + fabs(d[m + 1]);
          if (fabs(e[m]) <= 2.220446049250313e-16 * fmax(dd, tnorm)) break;
        }
        s_lo = 1;
        s_hi = 0;  // empty: converged
        if (m != l && iter >= 30) {
          atomicOr(flag + 3, 1);
        } else if (m != l) {
          // shift from the leading 2 x 2 block, then chase the bulge upward from m
          double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
          double r = hypot(g, 1.0);
          g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
          double sn = 1.0, cs = 1.0, pp = 0.0;
          int i = m - 1;
          bool split = false;
          for (; i >= l; --i) {
            const double f = sn * e[i], b = cs * e[i];
            r = hypot(f, g);
            e[i + 1] = r;
            if (r == 0.0) {  // the rotation would be undefined: T splits here
              d[i + 1] -= pp;
              e[m] = 0.0;
              split = true;
              break;
            }
            sn = f / r;
            cs = g / r;
            g = d[i + 1] - pp;
            r = (d[i] - g) * sn + 2.0 * cs * b;
            pp = sn * r;
            d[i + 1] = g + pp;
            g = cs * r - b;
            rc[i] = cs;
            rs[i] = sn;
          }
          if (!split) {
            d[l] -= pp;
            e[l] = g;
            e[m] = 0.0;
          }
          s_hi = m - 1;
          s_lo = split ? i + 1 : l;
        }
      }
      __syncthreads();
      const int lo = s_lo, hi = s_hi;
      if (lo > hi) {
        __syncthreads();
        break;  // uniform: eigenvalue l converged (or gave up)
      }
      // each row of Z through the rotations hi..lo; column i+1 is final after
      // rotation i, column i carries into the next one.  Chunks of QL_CH
      // loads are issued together instead of one dependent load per rotation.
      for (int r = t; r < n; r += blockDim.x) {
        double* zr = Z + (size_t)r * ld;
        double carry = zr[hi + 1];
        for (int i = hi; i >= lo; i -= QL_CH) {
          const int cnt = i - lo + 1 < QL_CH ? i - lo + 1 : QL_CH;
          double buf[QL_CH];
#pragma unroll
          for (int c = 0; c < QL_CH; ++c)
            if (c < cnt) buf[c] = zr[i - c];
#pragma unroll
          for (int c = 0; c < QL_CH; ++c)
            if (c < cnt) {
              const int ii = i - c;
              const double a = buf[c];
              buf[c] = rs[ii] * a + rc[ii] * carry;
              carry = rc[ii] * a - rs[ii] * carry;
            }
#pragma unroll
          for (int c = 0; c < QL_CH; ++c)
            if (c < cnt) zr[i - c + 1] = buf[c];
        }
        zr[lo] = carry;
      }
      __syncthreads();
    }
  }
  for (int i = t; i < n; i += blockDim.x) A[(size_t)i * ld + i] = d[i];
  __syncthreads();
}

// One problem per workgroup.  Scratch per problem: 4 ld^2 doubles.
__global__ __launch_bounds__(NT) void rr_kernel(const int32_t* m_arr, int ld, const double* H, const double* S,
                                                int nev, double drop_tol, int allow_svqb, double* evals, double* Vout,
                                                int32_t* rank_out, double* scratch, int* flag) {
  __shared__ double red[NT];
  __shared__ double sh_c[512], sh_s[512], sh_v[512], sh_w[512], sh_d[512], sh_e[512], sh_t[512];
  __shared__ double piv[512];
  __shared__ int sh_ord[512];
  __shared__ int use_chol, rank_sh;
  const int b = blockIdx.x, t = threadIdx.x;
  const int m = m_arr[b];
  const size_t L2 = (size_t)ld * ld;
  const double* Hb = H + b * L2;
  const double* Sb = S + b * L2;
  double* L = scratch + (size_t)b * 4 * L2;  // Cholesky factor / basis B
  double* C = L + L2;                         // reduced matrix
  double* Y = C + L2;                         // eigenvectors of C
  double* T = Y + L2;                         // temporary
  // symmetrised copies
  for (int i = t; i < m * m; i += NT) {
    const int r = i / m, c = i - r * m;
    L[r * ld + c] = 0.5 * (Sb[r * ld + c] + Sb[c * ld + r]);
    T[r * ld + c] = 0.5 * (Hb[r * ld + c] + Hb[c * ld + r]);
  }
  __syncthreads();
  double dmax = 0;
  for (int i = t; i < m; i += NT) dmax = fmax(dmax, L[i * ld + i]);
  red[t] = dmax;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  dmax = red[0];
  __syncthreads();
  if (t == 0) use_chol = 1;
  __syncthreads();
  // Cholesky in place (lower triangle of L), column by column
  // (the pivot's sum over k by wave 0's lanes; inner loops unrolled so that
  // their independent loads are in flight together)
  for (int j = 0; j < m; ++j) {
    if (t < 64) {
      double part = 0;
      for (int k = t; k < j; k += 64) part += L[j * ld + k] * L[j * ld + k];
      const double d = L[j * ld + j] - wave_sum64(part);
      if (t == 0) {
        if (!(d > drop_tol * dmax)) use_chol = 0;
        piv[j] = d > 0 ? sqrt(d) : 0.0;
        L[j * ld + j] = piv[j];
      }
    }
    __syncthreads();
    if (!use_chol) break;
    for (int i = j + 1 + t; i < m; i += NT) {
      double s = L[i * ld + j];
#pragma unroll 8
      for (int k = 0; k < j; ++k) s -= L[i * ld + k] * L[j * ld + k];
      L[i * ld + j] = s / piv[j];
    }
    __syncthreads();
  }
  int r;
  if (use_chol) {
    r = m;
    // C = L^{-1} Hs L^{-T}: X = L^{-1} Hs (forward substitution per column), then C = L^{-1} X^T
    for (int c = t; c < m; c += NT) {
      for (int i = 0; i < m; ++i) {
        double s = T[i * ld + c];
#pragma unroll 8
        for (int k = 0; k < i; ++k) s -= L[i * ld + k] * Y[k * ld + c];
        Y[i * ld + c] = s / L[i * ld + i];
      }
    }
    __syncthreads();
    for (int c = t; c < m; c += NT) {
      for (int i = 0; i < m; ++i) {
        double s = Y[c * ld + i];  // X^T[i][c] = X[c][i]
#pragma unroll 8
        for (int k = 0; k < i; ++k) s -= L[i * ld + k] * C[k * ld + c];
        C[i * ld + c] = s / L[i * ld + i];
      }
    }
    __syncthreads();
    // symmetrise
    for (int i = t; i < m * m; i += NT) {
      const int a = i / m, c = i - a * m;
      if (a < c) {
        const double v = 0.5 * (C[a * ld + c] + C[c * ld + a]);
        C[a * ld + c] = v;
        C[c * ld + a] = v;
      }
    }
    __syncthreads();
  } else {
    if (!allow_svqb) {
      if (t == 0) atomicOr(flag + 1, 1);
      for (int i = t; i < nev; i += NT) evals[b * nev + i] = NAN;
      if (t == 0) rank_out[b] = 0;
      return;
    }
    // SVQB: S = U Sigma U^T (Jacobi), keep sigma > drop_tol sigma_max, B = U_r Sigma_r^{-1/2}
    for (int i = t; i < m * m; i += NT) {
      const int a = i / m, c = i - a * m;
      C[a * ld + c] = 0.5 * (Sb[a * ld + c] + Sb[c * ld + a]);
    }
    __syncthreads();
    sym_eig(C, Y, m, ld, sh_c, sh_s, sh_v, sh_w, sh_d, sh_e, sh_t, red, flag);
    // eigenvalues on the diagonal of C; select kept columns (in index order)
    if (t == 0) {
      double smax = 0;
      for (int i = 0; i < m; ++i) smax = fmax(smax, C[i * ld + i]);
      int cnt = 0;
      for (int i = 0; i < m; ++i)
        if (C[i * ld + i] > drop_tol * smax) {
          sh_ord[cnt] = i;
          piv[cnt] = 1.0 / sqrt(C[i * ld + i]);
          ++cnt;
        }
      rank_sh = cnt;
    }
    __syncthreads();
    r = rank_sh;
    // L <- B (m x r)
    for (int i = t; i < m * r; i += NT) {
      const int a = i / r, j = i - a * r;
      L[a * ld + j] = Y[a * ld + sh_ord[j]] * piv[j];
    }
    __syncthreads();
    // Y <- Hs B (m x r), then C <- B^T Y (r x r)
    for (int i = t; i < m * r; i += NT) {
      const int a = i / r, j = i - a * r;
      double s = 0;
      for (int k = 0; k < m; ++k) s += T[a * ld + k] * L[k * ld + j];
      Y[a * ld + j] = s;
    }
    __syncthreads();
    for (int i = t; i < r * r; i += NT) {
      const int a = i / r, j = i - a * r;
      double s = 0;
      for (int k = 0; k < m; ++k) s += L[k * ld + a] * Y[k * ld + j];
      C[a * ld + j] = s;
    }
    __syncthreads();
    for (int i = t; i < r * r; i += NT) {
      const int a = i / r, c = i - a * r;
      if (a < c) {
        const double v = 0.5 * (C[a * ld + c] + C[c * ld + a]);
        C[a * ld + c] = v;
        C[c * ld + a] = v;
      }
    }
    __syncthreads();
  }
  // eigen-decomposition of the reduced r x r problem: C -> diag, Y eigenvectors
  sym_eig(C, Y, r, ld, sh_c, sh_s, sh_v, sh_w, sh_d, sh_e, sh_t, red, flag);
  // order eigenvalues ascending
  if (t == 0) {
    for (int i = 0; i < r; ++i) sh_ord[i] = i;
    for (int i = 1; i < r; ++i) {  // insertion sort (r <= 512)
      const int x = sh_ord[i];
      const double vx = C[x * ld + x];
      int j = i - 1;
      while (j >= 0 && C[sh_ord[j] * ld + sh_ord[j]] > vx) {
        sh_ord[j + 1] = sh_ord[j];
        --j;
      }
      sh_ord[j + 1] = x;
    }
    rank_out[b] = r;
  }
  __syncthreads();
  const int ne = nev < r ? nev : r;
  for (int i = t; i < nev; i += NT) evals[b * nev + i] = i < ne ? C[sh_ord[i] * ld + sh_ord[i]] : NAN;
  // back-transform: V = B Y  (B = L^{-T} in the Cholesky case)
  double* Vb = Vout + (size_t)b * ld * nev;
  if (use_chol) {
    // solve L^T V = Y_sel  (back substitution per column)
    for (int j = t; j < ne; j += NT) {
      const int col = sh_ord[j];
      for (int i = m - 1; i >= 0; --i) {
        double s = Y[i * ld + col];
#pragma unroll 8
        for (int k = i + 1; k < m; ++k) s -= L[k * ld + i] * T[k * ld + j];
        T[i * ld + j] = s / L[i * ld + i];
      }
    }
  } else {
    for (int e = t; e < m * ne; e += NT) {
      const int i = e / ne, j = e - i * ne;
      const int col = sh_ord[j];
      double s = 0;
      for (int k = 0; k < r; ++k) s += L[i * ld + k] * Y[k * ld + col];
      T[i * ld + j] = s;
    }
  }
  __syncthreads();
  // sign convention: entry of largest magnitude positive
  for (int j = t; j < ne; j += NT) {
    int im = 0;
    double vm = 0;
    for (int i = 0; i < m; ++i)
      if (fabs(T[i * ld + j]) > vm) {
        vm = fabs(T[i * ld + j]);
        im = i;
      }
    piv[j] = T[im * ld + j] < 0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int e = t; e < ld * nev; e += NT) {
    const int i = e / nev, j = e - i * nev;
    Vb[i * nev + j] = (i < m && j < ne) ? piv[j] * T[i * ld + j] : 0.0;
  }
}

hipError_t launch_rr(int batch, const int32_t* d_m, int ld, const double* H, const double* S, int nev, double drop_tol,
                     int allow_svqb, double* evals, double* V, int32_t* rank, double* scratch, int* flag,
                     hipStream_t s) {
  hipLaunchKernelGGL(rr_kernel, dim3(batch), dim3(NT), 0, s, d_m, ld, H, S, nev, drop_tol, allow_svqb, evals, V, rank,
                     scratch, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------- QR gauge move
// Per state z (one workgroup of 4 wave64s): the node tensor viewed as the
// matrix A[r][j] = X[z*size + roff[r] + j*cstride] (rows = all other legs,
// columns = the leg toward the new centre), Householder QR in double with
// diag(R) >= 0.  Q overwrites the tensor; R (n x n) goes to Rout[z]; m >= n.
// For each reflector the dot products with all remaining columns are done at
// once: columns are dealt to the 4 waves, rows to the 64 lanes, each dot is a
// wave reduction, so a reflector costs two workgroup barriers.
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void qr_kernel(T* X, int64_t size, const int32_t* roff, int m, int n,
                                                 int64_t cstride, double* work, double* Rout, int* flag) {
  __shared__ double red[256];
  __shared__ double wdot[512];
  __shared__ double sh_tau, sh_alpha;
  const int z = blockIdx.x, t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  T* Xz = X + (int64_t)z * size;
  double* A = work + (size_t)z * ((size_t)m * n + (size_t)m * n);  // m x n working copy (column-major)
  double* Vh = A + (size_t)m * n;                                  // Householder vectors (column-major)
  double* tauv = Rout + (size_t)gridDim.x * n * n + (size_t)z * n;  // tau per reflector
  for (int i = t; i < m * n; i += 256) {
    const int j = i / m, r = i - j * m;
    A[i] = (double)Xz[roff[r] + (int64_t)j * cstride];
  }
  __syncthreads();
  double* R = Rout + (size_t)z * n * n;
  for (int k = 0; k < n; ++k) {
    const double* a = A + (size_t)k * m;
    double ss = 0;
    for (int i = k + t; i < m; i += 256) ss += a[i] * a[i];
    ss = block_sum(ss, red);
    const double nrm = sqrt(ss);
    double* v = Vh + (size_t)k * m;
    if (t == 0) {
      const double x0 = a[k];
      const double alpha = nrm == 0.0 ? 0.0 : (x0 >= 0 ? -nrm : nrm);
      const double v0 = x0 - alpha;
      const double vn2 = ss - x0 * x0 + v0 * v0;
      sh_tau = vn2 > 0 ? 2.0 / vn2 : 0.0;
      sh_alpha = alpha;
      tauv[k] = sh_tau;
    }
    __syncthreads();
    for (int i = t; i < m; i += 256) v[i] = i < k ? 0.0 : (i == k ? a[k] - sh_alpha : a[i]);
    __syncthreads();
    // w_j = v . a_j for j = k..n-1 (columns dealt to waves, rows to lanes)
    for (int j = k + wv; j < n; j += 4) {
      const double* aj = A + (size_t)j * m;
      double d = 0;
      for (int i = k + lane; i < m; i += 64) d += v[i] * aj[i];
      d = wave_sum(d);
      if (lane == 0) wdot[j] = d;
    }
    __syncthreads();
    const double tau = sh_tau;
    for (int e = t; e < (n - k) * (m - k); e += 256) {
      const int jj = e / (m - k), i = k + (e - jj * (m - k));
      const int j = k + jj;
      A[(size_t)j * m + i] -= tau * wdot[j] * v[i];
    }
    __syncthreads();
  }
  // R (upper triangle of A)
  for (int i = t; i < n * n; i += 256) {
    const int r = i / n, c = i - r * n;
    R[i] = (c >= r) ? A[(size_t)c * m + r] : 0.0;
  }
  __syncthreads();
  // Q = H_0 ... H_{n-1} applied to the first n unit columns; build in A
  for (int i = t; i < m * n; i += 256) {
    const int j = i / m, r = i - j * m;
    A[i] = (r == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = n - 1; k >= 0; --k) {
    const double* v = Vh + (size_t)k * m;
    const double tau = tauv[k];
    for (int j = wv; j < n; j += 4) {
      const double* qj = A + (size_t)j * m;
      double d = 0;
      for (int i = k + lane; i < m; i += 64) d += v[i] * qj[i];
      d = wave_sum(d);
      if (lane == 0) wdot[j] = d;
    }
    __syncthreads();
    for (int e = t; e < n * (m - k); e += 256) {
      const int j = e / (m - k), i = k + (e - j * (m - k));
      A[(size_t)j * m + i] -= tau * wdot[j] * v[i];
    }
    __syncthreads();
  }
  // sign fix: diag(R) >= 0
  __shared__ double sg[512];
  for (int i = t; i < n; i += 256) sg[i] = R[i * n + i] < 0 ? -1.0 : 1.0;
  __syncthreads();
  for (int i = t; i < n * n; i += 256) {
    const int r = i / n;
    R[i] *= sg[r];
  }
  for (int i = t; i < m * n; i += 256) {
    const int j = i / m, r = i - j * m;
    const double q = A[i] * sg[j];
    if (!isfinite(q)) atomicOr(flag, 1);
    Xz[roff[r] + (int64_t)j * cstride] = (T)q;
  }
}

// Householder QR with the working matrix resident in LDS (dynamic shared
// memory, FP64): column-major A (m x n); reflector k is stored in place below
// the diagonal normalised to v_k = 1 (tau scaled to match), R is saved to a
// small separate array, and Q is formed in place by backward accumulation of
// the reflectors (each column finished as -tau v below, 1 - tau on, 0 above
// the diagonal).  One workgroup per state, one barrier per reflector, with
// look-ahead: while waves 1..15 apply reflector k to columns k+2.. (dot product
// as a wave sum, then the update), wave 0 applies it to column k+1 and at once
// builds reflector k+1 from that column, which no other wave touches in the
// step.  The Q formation mirrors it: wave 0 finishes column i+1 as a column
// of Q and applies reflector i to it while the other waves take columns i+2..
// The sign fix makes diag(R) >= 0 as in the global-memory kernel above.
// Nodes whose m x n doubles do not fit go through the TSQR kernels below,
// which factor row blocks with the same LDS routine, and the global-memory
// kernel serves only shapes that TSQR cannot block.

#define QR_NT 1024  // threads of the LDS-resident QR (16 waves: more columns in flight per reflector)
#define QR_NW (QR_NT / 64)
#define QR_QG 8  // loads of a thread in flight together when a matrix is gathered from or scattered to a node

// A[j*rows + i] = Xz[roff[r0 + i] + j*cstride] in double (i < rows, j < n):
// a thread loads the row offsets of QR_QG elements, then the QR_QG elements,
// so that its loads overlap instead of waiting on one dependent pair at a time
template <typename T>
__device__ __forceinline__ void qr_gather(double* A, const T* Xz, const int32_t* roff, int r0, int rows, int n,
                                          int64_t cstride) {
  const int tot = rows * n;
  for (int e0 = threadIdx.x; e0 < tot; e0 += QR_QG * QR_NT) {
    // indices past the end are clamped to the last element, so every load is
    // unconditional (no branch between them) and only the stores are masked
    int64_t off[QR_QG];
#pragma unroll
    for (int u = 0; u < QR_QG; ++u) {
      const int e = min(e0 + u * QR_NT, tot - 1), j = e / rows, i = e - j * rows;
      off[u] = (int64_t)roff[r0 + i] + (int64_t)j * cstride;
    }
    T v[QR_QG];
#pragma unroll
    for (int u = 0; u < QR_QG; ++u) v[u] = Xz[off[u]];
#pragma unroll
    for (int u = 0; u < QR_QG; ++u)
      if (e0 + u * QR_NT < tot) A[e0 + u * QR_NT] = (double)v[u];
  }
}

// Householder QR of the m x n (m >= n) column-major matrix A in LDS by the
// whole workgroup.  On entry Rl (n x n, row-major) is zero; on return A holds
// the explicit Q and Rl the upper-triangular R, both before any sign fix;
// tau (n doubles) is scratch.
// ITM > 0: every row loop of a lane has at most ITM iterations (m <= 64 ITM),
// unrolled so that a lane's LDS loads are all in flight before its FMAs;
// ITM = 0: runtime-bounded loops.
template <int ITM>
__device__ __forceinline__ void qr_lds_factor(double* A, double* Rl, double* tau, int m, int n) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  constexpr int IT = ITM > 0 ? ITM : 1;
  const int nit = ITM > 0 ? ITM : (m + 63) / 64;  // iterations of the runtime form
  // y_i -= d v_i and d = sum v_i y_i over rows i = s + lane + 64 it (< m), with
  // the v rows loaded once per reflector
  auto dot_update = [&](const double* v, double* y, int s, int kd, double tk) {
    if constexpr (ITM > 0) {
      double vv[IT], yv[IT];
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int i = s + lane + 64 * it;
        vv[it] = i < m ? v[i] : 0.0;
        yv[it] = i < m ? y[i] : 0.0;
      }
      double d = lane == 0 ? y[kd] : 0.0;
#pragma unroll
      for (int it = 0; it < IT; ++it) d += vv[it] * yv[it];
      d = tk * wave_sum_dpp(d);
      if (lane == 0) y[kd] -= d;
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int i = s + lane + 64 * it;
        if (i < m) y[i] = yv[it] - d * vv[it];
      }
    } else {
      double d = lane == 0 ? y[kd] : 0.0;
      for (int i = s + lane; i < m; i += 64) d += v[i] * y[i];
      d = tk * wave_sum_dpp(d);
      if (lane == 0) y[kd] -= d;
      for (int i = s + lane; i < m; i += 64) y[i] -= d * v[i];
    }
  };
  (void)nit;
  // reflector k from column k (rows k..m-1), by one wave: v = (1, a[k+1..] / v0),
  // tau' = 2 v0^2 / |x - alpha e_k|^2; each lane reads the rows i = k + lane + 64 it
  auto build = [&](int k) {
    double* a = A + (size_t)k * m;
    double xv[IT];
    double ss = 0;
    if constexpr (ITM > 0) {
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int i = k + lane + 64 * it;
        xv[it] = i < m ? a[i] : 0.0;
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) ss += xv[it] * xv[it];
    } else {
      for (int i = k + lane; i < m; i += 64) ss += a[i] * a[i];
    }
    ss = wave_sum_dpp(ss);
    const double x0 = a[k], nrm = sqrt(ss);
    const double alpha = nrm == 0.0 ? 0.0 : (x0 >= 0 ? -nrm : nrm);
    const double v0 = x0 - alpha;
    const double vn2 = ss - x0 * x0 + v0 * v0;
    const double inv = v0 != 0.0 ? 1.0 / v0 : 0.0;
    if constexpr (ITM > 0) {
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int i = k + lane + 64 * it;
        if (i > k && i < m) a[i] = xv[it] * inv;
      }
    } else {
      for (int i = k + 1 + lane; i < m; i += 64) a[i] *= inv;
    }
    if (lane == 0) {
      tau[k] = (vn2 > 0 && v0 != 0.0) ? 2.0 * v0 * v0 / vn2 : 0.0;
      Rl[k * n + k] = alpha;
    }
  };
  // ITM > 0, one wave: reflector k applied to column k+1 (y), then reflector
  // k+1 built from the updated column while it is still in registers (the
  // same rows per lane as dot_update and build, so the same arithmetic)
  auto update_build = [&](const double* v, double* y, int k, double tk) {
    const int s = k + 1;
    double vv[IT], xv[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = s + lane + 64 * it;
      vv[it] = i < m ? v[i] : 0.0;
      xv[it] = i < m ? y[i] : 0.0;
    }
    double d = lane == 0 ? y[k] : 0.0;
#pragma unroll
    for (int it = 0; it < IT; ++it) d += vv[it] * xv[it];
    d = tk * wave_sum_dpp(d);
    if (lane == 0) y[k] -= d;
    double ss = 0;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      xv[it] = xv[it] - d * vv[it];
      ss += xv[it] * xv[it];
    }
    ss = wave_sum_dpp(ss);
    const double x0 = lane_value(xv[0], 0), nrm = sqrt(ss);
    const double alpha = nrm == 0.0 ? 0.0 : (x0 >= 0 ? -nrm : nrm);
    const double v0 = x0 - alpha;
    const double vn2 = ss - x0 * x0 + v0 * v0;
    const double inv = v0 != 0.0 ? 1.0 / v0 : 0.0;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = s + lane + 64 * it;
      if (i < m) y[i] = i > s ? xv[it] * inv : xv[it];
    }
    if (lane == 0) {
      tau[s] = (vn2 > 0 && v0 != 0.0) ? 2.0 * v0 * v0 / vn2 : 0.0;
      Rl[s * n + s] = alpha;
    }
  };
  // ITM > 0, one wave: column i+1 (y, holding reflector i+1 below its
  // diagonal) finished as e_{i+1} - tn v_{i+1}, then reflector i (v, ti)
  // applied to it, in one pass over the rows
  auto finish_update = [&](const double* v, double* y, int i, double ti, double tn) {
    const int s = i + 1;
    double vv[IT], yv[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int r = s + lane + 64 * it;
      vv[it] = r < m ? v[r] : 0.0;
      yv[it] = r < m ? (r > s ? -tn * y[r] : 1.0 - tn) : 0.0;
    }
    double d = 0.0;
#pragma unroll
    for (int it = 0; it < IT; ++it) d += vv[it] * yv[it];
    d = ti * wave_sum_dpp(d);
    for (int r = lane; r < s; r += 64) y[r] = r == i ? -d : 0.0;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int r = s + lane + 64 * it;
      if (r < m) y[r] = yv[it] - d * vv[it];
    }
  };
  // LDS writes of this wave's lanes visible to its other lanes
  auto wave_lds_sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  };
  if (wv == 0) build(0);
  __syncthreads();
  for (int k = 0; k + 1 < n; ++k) {
    const double* a = A + (size_t)k * m;
    const double tk = tau[k];
    if (wv == 0) {
      if constexpr (ITM > 0) {
        update_build(a, A + (size_t)(k + 1) * m, k, tk);
      } else {
        dot_update(a, A + (size_t)(k + 1) * m, k + 1, k, tk);
        wave_lds_sync();
        build(k + 1);
      }
    } else {
      for (int j = k + 1 + wv; j < n; j += QR_NW - 1) dot_update(a, A + (size_t)j * m, k + 1, k, tk);
    }
    __syncthreads();
  }
  for (int e = t; e < n * n; e += QR_NT) {
    const int r = e / n, c = e - r * n;
    if (c > r) Rl[e] = A[(size_t)c * m + r];
  }
  __syncthreads();
  // Q in place: backward accumulation of the reflectors; column i is finished
  // as e_i - tau_i v_i once every dot with reflector i is done
  auto finish = [&](int i, int t0, int stride) {
    double* ai = A + (size_t)i * m;
    const double ti = tau[i];
    for (int r = t0; r < m; r += stride) ai[r] = r > i ? -ti * ai[r] : (r == i ? 1.0 - ti : 0.0);
  };
  for (int i = n - 2; i >= 0; --i) {
    const double* ai = A + (size_t)i * m;
    const double ti = tau[i];
    if (wv == 0) {
      if constexpr (ITM > 0) {
        finish_update(ai, A + (size_t)(i + 1) * m, i, ti, tau[i + 1]);
      } else {
        finish(i + 1, lane, 64);
        wave_lds_sync();
        dot_update(ai, A + (size_t)(i + 1) * m, i + 1, i, ti);
      }
    } else {
      for (int j = i + 1 + wv; j < n; j += QR_NW - 1) dot_update(ai, A + (size_t)j * m, i + 1, i, ti);
    }
    __syncthreads();
  }
  finish(0, t, QR_NT);
  __syncthreads();
}

template <typename T, int ITM>
__global__ __launch_bounds__(QR_NT) void qr_lds_kernel(T* X, int64_t size, const int32_t* roff, int m, int n,
                                                     int64_t cstride, double* Rout, int* flag) {
  extern __shared__ double sm[];
  double* A = sm;                  // m * n, column-major
  double* Rl = A + (size_t)m * n;  // n * n, row-major
  double* tau = Rl + (size_t)n * n;
  const int z = blockIdx.x, t = threadIdx.x;
  T* Xz = X + (int64_t)z * size;
  qr_gather(A, Xz, roff, 0, m, n, cstride);
  for (int i = t; i < n * n; i += QR_NT) Rl[i] = 0.0;
  __syncthreads();
  qr_lds_factor<ITM>(A, Rl, tau, m, n);
  // sign fix diag(R) >= 0, R out (row-major), Q back to the node tensor
  double* R = Rout + (size_t)z * n * n;
  for (int e = t; e < n * n; e += QR_NT) {
    const int r = e / n;
    R[e] = Rl[r * n + r] < 0 ? -Rl[e] : Rl[e];
  }
  const int tot = m * n;
  for (int e0 = t; e0 < tot; e0 += QR_QG * QR_NT) {
    int64_t off[QR_QG];
#pragma unroll
    for (int u = 0; u < QR_QG; ++u) {
      const int e = min(e0 + u * QR_NT, tot - 1), j = e / m, r = e - j * m;
      off[u] = (int64_t)roff[r] + (int64_t)j * cstride;
    }
#pragma unroll
    for (int u = 0; u < QR_QG; ++u) {
      const int e = e0 + u * QR_NT, j = e / m;
      if (e < tot) {
        const double q = Rl[j * n + j] < 0 ? -A[e] : A[e];
        if (!isfinite(q)) atomicOr(flag, 1);
        Xz[off[u]] = (T)q;
      }
    }
  }
}

// Register-resident form of the same Householder QR for m <= 64 ITM rows and
// n <= 16 CPW columns: wave w keeps columns w, w + 16, .. in registers (lane l
// holds rows l + 64 it), and only the reflectors go through LDS (v_k over
// rows > k, v_k[k] = 1 implied; tau_k; alpha_k = R[k][k] before the sign
// fix).  Factorisation step k: every wave reads v_k once and applies it to its
// columns j > k; the owner of column k+1 updates that column first and builds
// v_{k+1} from it at once, so a step costs one barrier and moves one column's
// worth of LDS reads per wave instead of every column's reads and writes.  Q
// by backward accumulation needs no barrier at all: column j of Q is
// H_0 .. H_{j-1} (e_j - tau_j v_j), and every reflector is in LDS by then, so
// each wave forms its own columns.
template <typename T, int ITM, int CPW>
__global__ __launch_bounds__(QR_NT) void qr_reg_kernel(T* X, int64_t size, const int32_t* roff, int m, int n,
                                                     int64_t cstride, double* Rout, int* flag) {
  extern __shared__ double sm[];
  double* V = sm;                   // V[k m + r]
  double* tau = V + (size_t)m * n;  // n
  double* rd = tau + n;             // n
  const int z = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  T* Xz = X + (int64_t)z * size;
  double col[CPW][ITM];
  int64_t ro[ITM];
#pragma unroll
  for (int it = 0; it < ITM; ++it) ro[it] = roff[min(lane + 64 * it, m - 1)];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int64_t jo = (int64_t)min(wv + QR_NW * c, n - 1) * cstride;
#pragma unroll
    for (int it = 0; it < ITM; ++it) col[c][it] = (double)Xz[ro[it] + jo];
  }
#pragma unroll
  for (int it = 0; it < ITM; ++it)
    if (lane + 64 * it >= m) {
#pragma unroll
      for (int c = 0; c < CPW; ++c) col[c][it] = 0.0;
    }
  // reflector k from the owner's column x (rows >= k): v = x / v0 below row k,
  // tau' = 2 v0^2 / |x - alpha e_k|^2, as in the LDS kernel
  auto build = [&](const double (&x)[ITM], int k) {
    double ss = 0.0, xk = 0.0;
#pragma unroll
    for (int it = 0; it < ITM; ++it) {
      const int r = lane + 64 * it;
      if (r >= k) ss += x[it] * x[it];
      if (it == (k >> 6)) xk = x[it];
    }
    ss = wave_sum_dpp(ss);
    const double x0 = lane_value(xk, k & 63), nrm = sqrt(ss);
    const double alpha = nrm == 0.0 ? 0.0 : (x0 >= 0 ? -nrm : nrm);
    const double v0 = x0 - alpha;
    const double vn2 = ss - x0 * x0 + v0 * v0;
    const double inv = v0 != 0.0 ? 1.0 / v0 : 0.0;
#pragma unroll
    for (int it = 0; it < ITM; ++it) {
      const int r = lane + 64 * it;
      if (r > k && r < m) V[(size_t)k * m + r] = x[it] * inv;
    }
    if (lane == 0) {
      tau[k] = (vn2 > 0 && v0 != 0.0) ? 2.0 * v0 * v0 / vn2 : 0.0;
      rd[k] = alpha;
    }
  };
  // v_k over this lane's rows (zero above row k)
  auto load_v = [&](double (&v)[ITM], int k) {
#pragma unroll
    for (int it = 0; it < ITM; ++it) {
      const int r = lane + 64 * it;
      v[it] = (r > k && r < m) ? V[(size_t)k * m + r] : (r == k ? 1.0 : 0.0);
    }
  };
  auto apply = [&](double (&y)[ITM], const double (&v)[ITM], double tk) {
    double d = 0.0;
#pragma unroll
    for (int it = 0; it < ITM; ++it) d += v[it] * y[it];
    d = tk * wave_sum_dpp(d);
#pragma unroll
    for (int it = 0; it < ITM; ++it) y[it] -= d * v[it];
  };
  if (wv == 0) build(col[0], 0);
  __syncthreads();
  for (int k = 0; k + 1 < n; ++k) {
    if (wv + QR_NW * (CPW - 1) > k) {  // some column of this wave is past k
      double v[ITM];
      load_v(v, k);
      const double tk = tau[k];
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int j = wv + QR_NW * c;
        if (j > k && j < n) {
          apply(col[c], v, tk);
          if (j == k + 1) build(col[c], k + 1);
        }
      }
    }
    __syncthreads();
  }
  // R (sign-fixed rows) from the owners' registers: rows above the diagonal
  // are final since their reflectors were applied
  double* R = Rout + (size_t)z * n * n;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int j = wv + QR_NW * c;
    if (j < n) {
#pragma unroll
      for (int it = 0; it < ITM; ++it) {
        const int r = lane + 64 * it;
        if (r < n) {
          const double val = r < j ? col[c][it] : (r == j ? rd[j] : 0.0);
          R[(size_t)r * n + j] = rd[r] < 0 ? -val : val;
        }
      }
    }
  }
  // Q: every owned column finished as e_j - tau_j v_j, then H_i for i < j
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int j = wv + QR_NW * c;
    if (j < n) {
      const double tj = tau[j];
#pragma unroll
      for (int it = 0; it < ITM; ++it) {
        const int r = lane + 64 * it;
        col[c][it] = (r > j && r < m) ? -tj * V[(size_t)j * m + r] : (r == j ? 1.0 - tj : 0.0);
      }
    }
  }
  for (int i = n - 2; i >= 0; --i) {
    if (wv + QR_NW * (CPW - 1) <= i) continue;
    double v[ITM];
    load_v(v, i);
    const double ti = tau[i];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int j = wv + QR_NW * c;
      if (j > i && j < n) apply(col[c], v, ti);
    }
  }
  // Q (sign-fixed columns) back to the node tensor
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int j = wv + QR_NW * c;
    if (j < n) {
      const double sg = rd[j] < 0 ? -1.0 : 1.0;
#pragma unroll
      for (int it = 0; it < ITM; ++it) {
        if (lane + 64 * it < m) {
          const double q = sg * col[c][it];
          if (!isfinite(q)) atomicOr(flag, 1);
          Xz[ro[it] + (int64_t)j * cstride] = (T)q;
        }
      }
    }
  }
}

// Tall-skinny QR (TSQR) for node matrices whose m x n doubles do not fit one
// workgroup's LDS: the rows are cut into P blocks of mb rows (the last block
// shorter, none below n rows).  Per state z the workspace W_z (2 m n doubles)
// holds the blocks' explicit Q_b (rows_b x n, column-major) at W_z + r0_b n,
// then the stacked R factors S ((P n) x n, column-major) at W_z + m n.
// Leaf: block b of state z factored in LDS with the kernel above.
template <typename T, int ITM>
__global__ __launch_bounds__(QR_NT) void tsqr_leaf_kernel(const T* X, int64_t size, const int32_t* roff, int m,
                                                        int n, int64_t cstride, int mb, int P, double* work) {
  extern __shared__ double sm[];
  const int b = blockIdx.x, z = blockIdx.y, t = threadIdx.x;
  const int r0 = b * mb, rows = min(mb, m - r0);
  double* A = sm;
  double* Rl = A + (size_t)rows * n;
  double* tau = Rl + (size_t)n * n;
  qr_gather(A, X + (int64_t)z * size, roff, r0, rows, n, cstride);
  for (int i = t; i < n * n; i += QR_NT) Rl[i] = 0.0;
  __syncthreads();
  qr_lds_factor<ITM>(A, Rl, tau, rows, n);
  double* Wz = work + (size_t)z * 2 * m * n;
  double* Qb = Wz + (size_t)r0 * n;
  for (int e = t; e < rows * n; e += QR_NT) Qb[e] = A[e];
  double* S = Wz + (size_t)m * n;
  const int ps = P * n;
  for (int e = t; e < n * n; e += QR_NT) {
    const int r = e / n, c = e - r * n;
    S[(size_t)c * ps + b * n + r] = Rl[e];  // zero below the diagonal
  }
}

// Root: S = Q2 R in LDS, diag(R) >= 0 by flipping rows of R and the matching
// columns of Q2; R to Rout[z] (row-major), Q2 over S.
template <int ITM>
__global__ __launch_bounds__(QR_NT) void tsqr_root_kernel(int m, int n, int P, double* work, double* Rout) {
  extern __shared__ double sm[];
  const int z = blockIdx.x, t = threadIdx.x, ps = P * n;
  double* A = sm;
  double* Rl = A + (size_t)ps * n;
  double* tau = Rl + (size_t)n * n;
  double* S = work + (size_t)z * 2 * m * n + (size_t)m * n;
  for (int e = t; e < ps * n; e += QR_NT) A[e] = S[e];
  for (int i = t; i < n * n; i += QR_NT) Rl[i] = 0.0;
  __syncthreads();
  qr_lds_factor<ITM>(A, Rl, tau, ps, n);
  double* R = Rout + (size_t)z * n * n;
  for (int e = t; e < n * n; e += QR_NT) {
    const int r = e / n;
    R[e] = Rl[r * n + r] < 0 ? -Rl[e] : Rl[e];
  }
  for (int e = t; e < ps * n; e += QR_NT) {
    const int j = e / ps;
    S[e] = Rl[j * n + j] < 0 ? -A[e] : A[e];
  }
}

// Apply: the rows of block b of the state's Q are Q_b times rows b n .. b n + n - 1
// of Q2; Q_b and that n x n slice staged in LDS, a thread per (row, QR_NC
// output columns), written into the node tensor.
#define QR_NC 8
template <typename T>
__global__ __launch_bounds__(QR_NT) void tsqr_apply_kernel(T* X, int64_t size, const int32_t* roff, int m, int n,
                                                         int64_t cstride, int mb, int P, const double* work,
                                                         int* flag) {
  extern __shared__ double sm[];
  const int b = blockIdx.x, z = blockIdx.y, t = threadIdx.x;
  const int r0 = b * mb, rows = min(mb, m - r0), ps = P * n;
  const double* Wz = work + (size_t)z * 2 * m * n;
  const double* Qb = Wz + (size_t)r0 * n;
  const double* Q2 = Wz + (size_t)m * n;
  double* sq = sm;                          // rows x n, column-major
  double* s2 = sq + (size_t)rows * n;       // n x n: s2[l n + j] = Q2[b n + l][j]
  const int tot = rows * n;
  for (int e0 = t; e0 < tot; e0 += QR_QG * QR_NT) {
    double v[QR_QG];
#pragma unroll
    for (int u = 0; u < QR_QG; ++u) v[u] = Qb[min(e0 + u * QR_NT, tot - 1)];
#pragma unroll
    for (int u = 0; u < QR_QG; ++u)
      if (e0 + u * QR_NT < tot) sq[e0 + u * QR_NT] = v[u];
  }
  for (int e = t; e < n * n; e += QR_NT) {
    const int l = e / n, j = e - l * n;
    s2[e] = Q2[(size_t)j * ps + b * n + l];
  }
  __syncthreads();
  T* Xz = X + (int64_t)z * size;
  const int nch = (n + QR_NC - 1) / QR_NC;
  for (int w = t; w < rows * nch; w += QR_NT) {
    const int c = w / rows, i = w - c * rows, j0 = c * QR_NC;
    const int64_t ro = roff[r0 + i];
    double acc[QR_NC];
#pragma unroll
    for (int q = 0; q < QR_NC; ++q) acc[q] = 0.0;
    for (int l = 0; l < n; ++l) {
      const double a = sq[(size_t)l * rows + i];
#pragma unroll
      for (int q = 0; q < QR_NC; ++q) acc[q] += a * s2[l * n + min(j0 + q, n - 1)];
    }
#pragma unroll
    for (int q = 0; q < QR_NC; ++q) {
      if (j0 + q < n) {
        if (!isfinite(acc[q])) atomicOr(flag, 1);
        Xz[ro + (int64_t)(j0 + q) * cstride] = (T)acc[q];
      }
    }
  }
}

// Y[z][roff[r] + i*cstride] = sum_j R[z][i][j] X[z][roff[r] + j*cstride]   (into a separate buffer)
template <typename T>
__global__ void absorb_kernel(const T* X, int64_t size, const int32_t* roff, int m, int n, int64_t cstride,
                              const double* R, T* Y, int nz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)m * n;
  if (e >= per * nz) return;
  const int z = (int)(e / per);
  const int64_t rem = e - (int64_t)z * per;
  const int r = (int)(rem / n), i = (int)(rem - (int64_t)r * n);
  const T* Xz = X + (int64_t)z * size;
  const double* Rz = R + (size_t)z * n * n;
  double s = 0;
  for (int j = 0; j < n; ++j) s += Rz[i * n + j] * (double)Xz[roff[r] + (int64_t)j * cstride];
  Y[(int64_t)z * size + roff[r] + (int64_t)i * cstride] = (T)s;
}

// Row-wise absorption for bonds n <= 48: a workgroup takes 64 whole rows of
// one state; lane l of wave w holds row r0 + l and columns w, w + 4, .., so
// that a wave's loads run along consecutive rows.  The rows are staged in LDS
// (column-major), and after the barrier each thread computes its outputs
// Y[r][i] = sum_j R[i][j] X[r][j] (sum over j in order, as in the element-wise
// kernel) and writes them over its elements: every element of a row is read
// before any of them is written, so the kernel may work in place (Y == X).
// All loads of a thread are issued unconditionally (indices clamped) so they
// overlap.
#define ABS_NMAX 48
#define ABS_RB 64
template <typename T>
__global__ __launch_bounds__(256) void absorb_rows_kernel(const T* X, int64_t size, const int32_t* roff, int m, int n,
                                                          int64_t cstride, const double* R, T* Y) {
  __shared__ double sR[ABS_NMAX * ABS_NMAX];
  __shared__ double sx[ABS_NMAX * ABS_RB];  // sx[j * 64 + row]
  constexpr int QM = ABS_NMAX / 4;
  const int z = blockIdx.y, t = threadIdx.x, lr = t & 63, w = t >> 6;
  const int r = blockIdx.x * ABS_RB + lr;
  const bool act = r < m;
  const double* Rz = R + (size_t)z * n * n;
  for (int e = t; e < n * n; e += 256) sR[e] = Rz[e];
  const int64_t base = (int64_t)z * size + (int64_t)roff[act ? r : m - 1];
  T v[QM];
#pragma unroll
  for (int q = 0; q < QM; ++q) v[q] = X[base + (int64_t)min(w + 4 * q, n - 1) * cstride];
#pragma unroll
  for (int q = 0; q < QM; ++q)
    if (w + 4 * q < n) sx[(w + 4 * q) * ABS_RB + lr] = (double)v[q];
  __syncthreads();
  if (!act) return;
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    const int i = w + 4 * q;
    if (i < n) {
      const double* rr = sR + i * n;
      double sacc = 0;
      for (int j = 0; j < n; ++j) sacc += rr[j] * sx[j * ABS_RB + lr];
      Y[base + (int64_t)i * cstride] = (T)sacc;
    }
  }
}

template <typename T>
static hipError_t qr_t(void* X, int64_t size, const int32_t* roff, int m, int n, int64_t cstride, double* work,
                       double* R, int nz, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(qr_kernel<T>, dim3(nz), dim3(256), 0, s, (T*)X, size, roff, m, n, cstride, work, R, flag);
  return hipGetLastError();
}

// LDS budget of the resident-matrix QR (the CU has 160 KiB)
static constexpr size_t QR_LDS_MAX = 150 * 1024;

// f(std::integral_constant<int, ITM>) for the smallest unrolled row-loop
// bound ITM that covers `rows` (0: the runtime-bounded form)
template <typename F>
static bool with_itm(int rows, F&& f) {
  const int need = (rows + 63) / 64;  // row iterations of a lane
  if (need <= 1) return f(std::integral_constant<int, 1>{});
  if (need <= 2) return f(std::integral_constant<int, 2>{});
  if (need <= 3) return f(std::integral_constant<int, 3>{});
  if (need <= 4) return f(std::integral_constant<int, 4>{});
  if (need <= 6) return f(std::integral_constant<int, 6>{});
  if (need <= 9) return f(std::integral_constant<int, 9>{});
  if (need <= 12) return f(std::integral_constant<int, 12>{});
  if (need <= 16) return f(std::integral_constant<int, 16>{});
  return f(std::integral_constant<int, 0>{});
}

// TTN_QR_NOREG=1 keeps every resident matrix on the LDS kernel (for comparison)
static bool qr_reg_on() {
  static const bool on = getenv("TTN_QR_NOREG") == nullptr;
  return on;
}

// one-time opt-in of a kernel to QR_LDS_MAX bytes of dynamic LDS
static bool lds_opt_in(const void* fn) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)QR_LDS_MAX) == hipSuccess;
}

static size_t qr_lds_bytes(int m, int n) { return ((size_t)m * n + (size_t)n * n + (size_t)n) * sizeof(double); }

// the register-resident kernel for m <= 64 ITM (ITM <= 9) and n <= 16 CPW (CPW <= 3)
template <typename T, int ITM>
static bool qr_reg_it(void* X, int64_t size, const int32_t* roff, int m, int n, int64_t cstride, double* R, int nz,
                      int* flag, hipStream_t s) {
  const size_t bytes = ((size_t)m * n + 2 * (size_t)n) * sizeof(double);
  auto go = [&](auto C) {
    constexpr int CPW = decltype(C)::value;
    static const bool enabled = lds_opt_in(reinterpret_cast<const void*>(&qr_reg_kernel<T, ITM, CPW>));
    if (!enabled) return false;
    hipLaunchKernelGGL((qr_reg_kernel<T, ITM, CPW>), dim3(nz), dim3(QR_NT), bytes, s, (T*)X, size, roff, m, n,
                       cstride, R, flag);
    return hipGetLastError() == hipSuccess;
  };
  if (n <= 16) return go(std::integral_constant<int, 1>{});
  if (n <= 32) return go(std::integral_constant<int, 2>{});
  return go(std::integral_constant<int, 3>{});
}

static bool qr_reg_fits(int m, int n) { return m <= 64 * 9 && n <= 48 && qr_lds_bytes(m, n) <= QR_LDS_MAX; }

template <typename T>
static bool qr_reg(void* X, int64_t size, const int32_t* roff, int m, int n, int64_t cstride, double* R, int nz,
                   int* flag, hipStream_t s) {
  if (!qr_reg_fits(m, n)) return false;
  return with_itm(m, [&](auto I) {
    constexpr int ITM = decltype(I)::value;
    if constexpr (ITM == 0 || ITM > 9) {
      return false;
    } else {
      return qr_reg_it<T, ITM>(X, size, roff, m, n, cstride, R, nz, flag, s);
    }
  });
}

template <typename T>
static bool qr_lds(void* X, int64_t size, const int32_t* roff, int m, int n, int64_t cstride, double* R, int nz,
                   int* flag, hipStream_t s) {
  const size_t bytes = qr_lds_bytes(m, n);
  if (bytes > QR_LDS_MAX) return false;
  if (qr_reg_on() && qr_reg<T>(X, size, roff, m, n, cstride, R, nz, flag, s)) return true;
  return with_itm(m, [&](auto I) {
    constexpr int ITM = decltype(I)::value;
    static const bool enabled = lds_opt_in(reinterpret_cast<const void*>(&qr_lds_kernel<T, ITM>));
    if (!enabled) return false;
    hipLaunchKernelGGL((qr_lds_kernel<T, ITM>), dim3(nz), dim3(QR_NT), bytes, s, (T*)X, size, roff, m, n, cstride,
                       R, flag);
    return hipGetLastError() == hipSuccess;
  });
}

// Row blocking of the TSQR path for an m x n matrix too tall for qr_lds: the
// fewest blocks whose leaf factorisation and apply fit QR_LDS_MAX, every block
// at least n rows, and the stacked R factors of all blocks within one
// workgroup's LDS; P = 0 when the path does not apply.
struct TsqrPlan {
  int P = 0, mb = 0;
};

static TsqrPlan tsqr_plan(int m, int n) {
  TsqrPlan p;
  if (qr_lds_bytes(m, n) <= QR_LDS_MAX) return p;
  const size_t lim = QR_LDS_MAX / sizeof(double), nn = (size_t)n * n;
  if (nn + n >= lim) return p;
  const size_t mbmax = (lim - nn - n) / n;  // leaf: (mb n + n n + n) doubles; the apply stages mb n + n n
  if (mbmax < (size_t)n) return p;
  const int P = (int)(((size_t)m + mbmax - 1) / mbmax);
  const int mb = (m + P - 1) / P;
  if (P < 2 || m - (P - 1) * mb < n) return p;
  if (qr_lds_bytes(P * n, n) > QR_LDS_MAX) return p;
  p.P = P;
  p.mb = mb;
  return p;
}

// Uses W_z = work + z 2 m n: Q_b blocks (m n doubles) then S ((P n) n <= m n).
template <typename T>
static bool tsqr(void* X, int64_t size, const int32_t* roff, int m, int n, int64_t cstride, double* work, double* R,
                 int nz, int* flag, hipStream_t s) {
  const TsqrPlan p = tsqr_plan(m, n);
  if (p.P == 0) return false;
  const bool leaf = with_itm(p.mb, [&](auto I) {
    constexpr int ITM = decltype(I)::value;
    static const bool enabled = lds_opt_in(reinterpret_cast<const void*>(&tsqr_leaf_kernel<T, ITM>));
    if (!enabled) return false;
    hipLaunchKernelGGL((tsqr_leaf_kernel<T, ITM>), dim3(p.P, nz), dim3(QR_NT), qr_lds_bytes(p.mb, n), s,
                       (const T*)X, size, roff, m, n, cstride, p.mb, p.P, work);
    return hipGetLastError() == hipSuccess;
  });
  if (!leaf) return false;
  const bool root = with_itm(p.P * n, [&](auto I) {
    constexpr int ITM = decltype(I)::value;
    static const bool enabled = lds_opt_in(reinterpret_cast<const void*>(&tsqr_root_kernel<ITM>));
    if (!enabled) return false;
    hipLaunchKernelGGL((tsqr_root_kernel<ITM>), dim3(nz), dim3(QR_NT), qr_lds_bytes(p.P * n, n), s, m, n, p.P, work,
                       R);
    return hipGetLastError() == hipSuccess;
  });
  if (!root) return false;
  static const bool apply_ok = lds_opt_in(reinterpret_cast<const void*>(&tsqr_apply_kernel<T>));
  if (!apply_ok) return false;
  const size_t abytes = ((size_t)p.mb * n + (size_t)n * n) * sizeof(double);
  hipLaunchKernelGGL(tsqr_apply_kernel<T>, dim3(p.P, nz), dim3(QR_NT), abytes, s, (T*)X, size, roff, m, n, cstride,
                     p.mb, p.P, (const double*)work, flag);
  return hipGetLastError() == hipSuccess;
}

static bool qr_global_only() {
  static const bool g = getenv("TTN_QR_GLOBAL") != nullptr;
  return g;
}

const char* qr_path_name(int m, int n) {
  if (qr_global_only()) return "qr_kernel";
  if (qr_lds_bytes(m, n) <= QR_LDS_MAX) return qr_reg_on() && qr_reg_fits(m, n) ? "qr_reg_kernel" : "qr_lds_kernel";
  if (tsqr_plan(m, n).P > 0) return "tsqr_kernels";
  return "qr_kernel";
}

// The LDS-resident kernel when the matrix fits, else TSQR when its blocks do,
// else the global-memory kernel; a path whose launch fails falls through to
// the next.  The TSQR launches run only once the leaf launch succeeded, so a
// partial TSQR never precedes the global kernel on the same data: the leaf
// and root read the node and write only the workspace.
hipError_t launch_qr(int ctype, void* X, int64_t size, const int32_t* roff, int m, int n, int64_t cstride, double* work,
                     double* R, int nz, int* flag, hipStream_t s) {
  if (!qr_global_only()) {
    if (ctype == 0 ? qr_lds<double>(X, size, roff, m, n, cstride, R, nz, flag, s)
                   : qr_lds<float>(X, size, roff, m, n, cstride, R, nz, flag, s))
      return hipSuccess;
    if (ctype == 0 ? tsqr<double>(X, size, roff, m, n, cstride, work, R, nz, flag, s)
                   : tsqr<float>(X, size, roff, m, n, cstride, work, R, nz, flag, s))
      return hipSuccess;
  }
  if (ctype == 0) return qr_t<double>(X, size, roff, m, n, cstride, work, R, nz, flag, s);
  return qr_t<float>(X, size, roff, m, n, cstride, work, R, nz, flag, s);
}

static hipError_t absorb_rows(int ctype, const void* X, int64_t size, const int32_t* roff, int m, int n,
                              int64_t cstride, const double* R, void* Y, int nz, hipStream_t s) {
  const dim3 grid((unsigned)((m + ABS_RB - 1) / ABS_RB), (unsigned)nz);
  if (ctype == 0)
    hipLaunchKernelGGL(absorb_rows_kernel<double>, grid, dim3(256), 0, s, (const double*)X, size, roff, m, n,
                       cstride, R, (double*)Y);
  else
    hipLaunchKernelGGL(absorb_rows_kernel<float>, grid, dim3(256), 0, s, (const float*)X, size, roff, m, n, cstride,
                       R, (float*)Y);
  return hipGetLastError();
}

// The row-wise kernel reads a whole row before writing it and rows are
// disjoint, so it may write over its input (Y == X): no copy back.
bool absorb_in_place(int m, int n) {
  (void)m;
  return n <= ABS_NMAX;
}

hipError_t launch_absorb(int ctype, const void* X, int64_t size, const int32_t* roff, int m, int n, int64_t cstride,
                         const double* R, void* Y, int nz, hipStream_t s) {
  // row-wise kernel, in place, for every bond it covers; the element-wise
  // kernel for larger bonds
  if (n <= ABS_NMAX) return absorb_rows(ctype, X, size, roff, m, n, cstride, R, Y, nz, s);
  const int64_t tot = (int64_t)m * n * nz;
  const unsigned g = (unsigned)((tot + 255) / 256);
  if (ctype == 0)
    hipLaunchKernelGGL(absorb_kernel<double>, dim3(g), dim3(256), 0, s, (const double*)X, size, roff, m, n, cstride, R,
                       (double*)Y, nz);
  else
    hipLaunchKernelGGL(absorb_kernel<float>, dim3(g), dim3(256), 0, s, (const float*)X, size, roff, m, n, cstride, R,
                       (float*)Y, nz);
  return hipGetLastError();
}

// ---------------------------------------------------------------- norms / scaling
template <typename T>
__global__ __launch_bounds__(256) void norms2_kernel(const T* X, int64_t n, double* out) {
  __shared__ double red[256];
  const int z = blockIdx.x;
  const T* x = X + (int64_t)z * n;
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)x[i] * (double)x[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[z] = s;
}

template <typename T>
__global__ void scale_kernel(T* X, int64_t n, const double* sc, int nz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nz) return;
  const int z = (int)(e / n);
  X[e] = (T)((double)X[e] * sc[z]);
}

hipError_t launch_norms2(int ctype, const void* X, int64_t n, int nz, double* out, hipStream_t s) {
  if (ctype == 0) hipLaunchKernelGGL(norms2_kernel<double>, dim3(nz), dim3(256), 0, s, (const double*)X, n, out);
  else hipLaunchKernelGGL(norms2_kernel<float>, dim3(nz), dim3(256), 0, s, (const float*)X, n, out);
  return hipGetLastError();
}

hipError_t launch_scale(int ctype, void* X, int64_t n, int nz, const double* sc, hipStream_t s) {
  const unsigned g = (unsigned)((n * nz + 255) / 256);
  if (ctype == 0) hipLaunchKernelGGL(scale_kernel<double>, dim3(g), dim3(256), 0, s, (double*)X, n, sc, nz);
  else hipLaunchKernelGGL(scale_kernel<float>, dim3(g), dim3(256), 0, s, (float*)X, n, sc, nz);
  return hipGetLastError();
}

}  // namespace ttn

namespace ttn {

// out[ia[i]] = out[ib[i]] = vals[i]
__global__ void scatter2_kernel(int n, const int32_t* ia, const int32_t* ib, const double* vals, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[ia[i]] = vals[i];
  out[ib[i]] = vals[i];
}

__global__ void vscale_kernel(int n, const double* x, double a, double* y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// per state: norm of the node tensor, then scale it to unit norm
template <typename T>
__global__ __launch_bounds__(256) void normalize_kernel(T* X, int64_t n, double* norms) {
  __shared__ double red[256];
  const int z = blockIdx.x;
  T* x = X + (int64_t)z * n;
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)x[i] * (double)x[i];
  s = block_sum(s, red);
  const double nr = sqrt(s);
  const double inv = nr > 0 ? 1.0 / nr : 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) x[i] = (T)((double)x[i] * inv);
  if (threadIdx.x == 0 && norms) norms[z] = nr;
}

hipError_t launch_scatter2(int n, const int32_t* ia, const int32_t* ib, const double* vals, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter2_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, ia, ib, vals, out);
  return hipGetLastError();
}

hipError_t launch_vscale(int n, const double* x, double a, double* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(vscale_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, x, a, y);
  return hipGetLastError();
}

hipError_t launch_normalize(int ctype, void* X, int64_t n, int nz, double* norms, hipStream_t s) {
  if (ctype == 0) hipLaunchKernelGGL(normalize_kernel<double>, dim3(nz), dim3(256), 0, s, (double*)X, n, norms);
  else hipLaunchKernelGGL(normalize_kernel<float>, dim3(nz), dim3(256), 0, s, (float*)X, n, norms);
  return hipGetLastError();
}

}  // namespace ttn
