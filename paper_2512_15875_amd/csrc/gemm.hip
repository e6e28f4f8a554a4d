// Offset-table GEMM on the CDNA4 matrix cores (gfx950).
//
// Every stage of a tensor-network contraction (environment update, H_eff
// product, diagonal) is a batched GEMM  C[z][m][n] = sum_k A[z][m][k] B[z][k][n]
// whose row, column and contraction indices are *groups* of tensor legs.  The
// address of an element is base(z) + row_off[m] + col_off[k] for A (likewise
// for B and C), with the offset tables precomputed on the host per stage, so a
// single kernel serves every leg permutation without transposes in HBM.
//
// Tiles: a 256-thread workgroup (4 wave64s in a 2x2 grid) owns a BM x BN tile
// of C; operands are staged through double-buffered LDS in BK-deep slices.
//   f64 : v_mfma_f64_16x16x4_f64  (A[l%16][l/16], B[l/16][l%16], D[l/16+4i][l%16])
//   f32 : v_mfma_f32_16x16x4_f32  (same inputs,                  D[4(l/16)+i][l%16])
//   bf16: v_mfma_f32_16x16x32_bf16 (8 consecutive k per lane,      D[4(l/16)+i][l%16])
// The bf16 form reads FP32 tensors and rounds to bfloat16 when staging to LDS.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ttn {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct KOp {
  const void* base;
  const int32_t* tab;
  int64_t bs;
  int mode;     // 0 shared, 1 table, 2 (z0+z), 3 z (chunk-local)
  int tab_max;  // valid table entries are [0, tab_max)
};

struct KArgs {
  KOp A, B, C, D;
  const int32_t *a_om, *a_ok, *b_ok, *b_on, *c_om, *c_on;
  const double* alpha;
  const double* shift;
  int M, N, K, z0, accum, tiles_n, has_d, d_const;
  int* flag;  // flag[2] is raised when a batch table holds an out-of-range index
};

__device__ __forceinline__ int64_t batch_off(const KOp& o, int z, int z0, int* flag) {
  switch (o.mode) {
    case 1: {
      int idx = o.tab[z0 + z];
      if (idx < 0 || idx >= o.tab_max) {  // clamp and report instead of reading out of bounds
        if (flag && threadIdx.x == 0) atomicOr(flag + 2, 1);
        idx = idx < 0 ? 0 : o.tab_max - 1;
      }
      return (int64_t)idx * o.bs;
    }
    case 2: return (int64_t)(z0 + z) * o.bs;
    case 3: return (int64_t)z * o.bs;
    default: return 0;
  }
}

template <int CT>
struct Types;
template <>
struct Types<0> {
  typedef double T;
  typedef double L;
  typedef doublex4 Acc;
};
template <>
struct Types<1> {
  typedef float T;
  typedef float L;
  typedef floatx4 Acc;
};
template <>
struct Types<2> {
  typedef float T;
  typedef __bf16 L;
  typedef floatx4 Acc;
};

template <int CT, int BM, int BN, int BK, bool AMF, bool BNF>
__global__ __launch_bounds__(256) void ogemm_kernel(KArgs g) {
  typedef typename Types<CT>::T T;
  typedef typename Types<CT>::L L;
  typedef typename Types<CT>::Acc Acc;
  constexpr int EA = BM * BK / 256;
  constexpr int EB = BN * BK / 256;
  constexpr int WTM = BM / 2, WTN = BN / 2;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  // LDS: f64/f32 keep k-major slices (a row of 16 m for one k is contiguous);
  // bf16 keeps m-major rows so that 8 consecutive k are one 16-byte read.
  constexpr int PADA = (CT == 2) ? 8 : 16 / (int)sizeof(L) * ((CT == 0) ? 1 : 4);
  constexpr int PADB = PADA;
  constexpr int LA = (CT == 2) ? BM * (BK + PADA) : BK * (BM + PADA);
  constexpr int LB = (CT == 2) ? BN * (BK + PADB) : BK * (BN + PADB);
  __shared__ L As[2][LA];
  __shared__ L Bs[2][LB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int z = blockIdx.y;
  const int tmi = blockIdx.x / g.tiles_n;
  const int tni = blockIdx.x - tmi * g.tiles_n;
  const int m0 = tmi * BM, n0 = tni * BN;
  const int M = g.M, N = g.N, K = g.K;

  const T* __restrict__ A = (const T*)g.A.base + batch_off(g.A, z, g.z0, g.flag);
  const T* __restrict__ B = (const T*)g.B.base + batch_off(g.B, z, g.z0, g.flag);

  // ---- fixed per-thread offsets
  int a_fix[AMF ? 1 : EA];
  int b_fix[BNF ? 1 : EB];
  if (AMF) {
    const int mg = m0 + tid % BM;
    a_fix[0] = (mg < M) ? g.a_om[mg] : -1;
  } else {
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int mg = m0 + tid / BK + i * (256 / BK);
      a_fix[i] = (mg < M) ? g.a_om[mg] : -1;
    }
  }
  if (BNF) {
    const int ng = n0 + tid % BN;
    b_fix[0] = (ng < N) ? g.b_on[ng] : -1;
  } else {
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int ng = n0 + tid / BK + i * (256 / BK);
      b_fix[i] = (ng < N) ? g.b_on[ng] : -1;
    }
  }

  T ra[EA], rb[EB];
  auto load = [&](int k0) {
    if (AMF) {
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int kg = k0 + tid / BM + i * (256 / BM);
        ra[i] = (a_fix[0] >= 0 && kg < K) ? A[a_fix[0] + g.a_ok[kg]] : (T)0;
      }
    } else {
      const int kg = k0 + tid % BK;
      const int ko = (kg < K) ? g.a_ok[kg] : -1;
#pragma unroll
      for (int i = 0; i < EA; ++i) ra[i] = (ko >= 0 && a_fix[i] >= 0) ? A[a_fix[i] + ko] : (T)0;
    }
    if (BNF) {
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int kg = k0 + tid / BN + i * (256 / BN);
        rb[i] = (b_fix[0] >= 0 && kg < K) ? B[b_fix[0] + g.b_ok[kg]] : (T)0;
      }
    } else {
      const int kg = k0 + tid % BK;
      const int ko = (kg < K) ? g.b_ok[kg] : -1;
#pragma unroll
      for (int i = 0; i < EB; ++i) rb[i] = (ko >= 0 && b_fix[i] >= 0) ? B[b_fix[i] + ko] : (T)0;
    }
  };
  auto aidx = [&](int m, int k) { return (CT == 2) ? m * (BK + PADA) + k : k * (BM + PADA) + m; };
  auto bidx = [&](int n, int k) { return (CT == 2) ? n * (BK + PADB) + k : k * (BN + PADB) + n; };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int ml = AMF ? tid % BM : tid / BK + i * (256 / BK);
      const int kl = AMF ? tid / BM + i * (256 / BM) : tid % BK;
      As[buf][aidx(ml, kl)] = (L)ra[i];
    }
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int nl = BNF ? tid % BN : tid / BK + i * (256 / BK);
      const int kl = BNF ? tid / BN + i * (256 / BN) : tid % BK;
      Bs[buf][bidx(nl, kl)] = (L)rb[i];
    }
  };

  Acc acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = Acc{0, 0, 0, 0};

  const int nk = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);
    if constexpr (CT == 2) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 32) {
        bf16x8 af[TM], bfr[TN];
#pragma unroll
        for (int a = 0; a < TM; ++a)
          af[a] = *(const bf16x8*)&As[buf][aidx(wm * WTM + a * 16 + (lane & 15), kk + 8 * (lane >> 4))];
#pragma unroll
        for (int b = 0; b < TN; ++b)
          bfr[b] = *(const bf16x8*)&Bs[buf][bidx(wn * WTN + b * 16 + (lane & 15), kk + 8 * (lane >> 4))];
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        L af[TM], bfr[TN];
#pragma unroll
        for (int a = 0; a < TM; ++a) af[a] = As[buf][aidx(wm * WTM + a * 16 + (lane & 15), kk + (lane >> 4))];
#pragma unroll
        for (int b = 0; b < TN; ++b) bfr[b] = Bs[buf][bidx(wn * WTN + b * 16 + (lane & 15), kk + (lane >> 4))];
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) {
            if constexpr (CT == 0)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bfr[b], acc[a][b], 0, 0, 0);
            else
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bfr[b], acc[a][b], 0, 0, 0);
          }
      }
    }
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  // ---- epilogue: C = alpha (acc - shift * D) (+ C)
  T* __restrict__ C = (T*)g.C.base + batch_off(g.C, z, g.z0, g.flag);
  const T* __restrict__ Dp = g.has_d ? (const T*)g.D.base + batch_off(g.D, z, g.z0, g.flag) : nullptr;
  const double alpha = g.alpha ? g.alpha[g.z0 + z] : 1.0;
  const double sh = g.shift ? g.shift[g.z0 + z] : 0.0;
#pragma unroll
  for (int a = 0; a < TM; ++a) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wm * WTM + a * 16 + ((CT == 0) ? ((lane >> 4) + 4 * i) : (4 * (lane >> 4) + i));
      const int mg = m0 + row;
      if (mg >= M) continue;
      const int64_t cm = g.c_om[mg];
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int ng = n0 + wn * WTN + b * 16 + (lane & 15);
        if (ng >= N) continue;
        const int64_t co = cm + g.c_on[ng];
        double v = (double)acc[a][b][i];
        if (Dp) v -= sh * (double)Dp[co];
        else if (g.d_const) v -= sh;
        v *= alpha;
        if (g.accum) v += (double)C[co];
        C[co] = (T)v;
      }
    }
  }
}

static KOp kop(const OpAddr& o, int default_mode) {
  KOp k;
  k.base = o.base;
  k.tab = o.tab;
  k.bs = o.bstride;
  k.tab_max = o.tab_max;
  if (o.shared) k.mode = 0;
  else if (o.tab) k.mode = 1;
  else if (o.local) k.mode = 3;
  else k.mode = default_mode;
  return k;
}

template <int CT, int BM, int BN, int BK>
static hipError_t launch_cfg(const GemmDesc& gd, KArgs& a, int nz, hipStream_t s) {
  const int tm = (gd.M + BM - 1) / BM, tn = (gd.N + BN - 1) / BN;
  a.tiles_n = tn;
  dim3 grid(tm * tn, nz);
  if (gd.a_mfast && gd.b_nfast) hipLaunchKernelGGL((ogemm_kernel<CT, BM, BN, BK, true, true>), grid, dim3(256), 0, s, a);
  else if (gd.a_mfast) hipLaunchKernelGGL((ogemm_kernel<CT, BM, BN, BK, true, false>), grid, dim3(256), 0, s, a);
  else if (gd.b_nfast) hipLaunchKernelGGL((ogemm_kernel<CT, BM, BN, BK, false, true>), grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((ogemm_kernel<CT, BM, BN, BK, false, false>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int CT>
static hipError_t launch_ct(const GemmDesc& gd, KArgs& a, int nz, hipStream_t s) {
  constexpr int BK = (CT == 2) ? 32 : 16;
  switch (gd.tile) {
    case 0: return launch_cfg<CT, 128, 128, BK>(gd, a, nz, s);
    case 1: return launch_cfg<CT, 64, 64, BK>(gd, a, nz, s);
    case 2: return launch_cfg<CT, 128, 64, BK>(gd, a, nz, s);
    case 3: return launch_cfg<CT, 64, 128, BK>(gd, a, nz, s);
    case 4: return launch_cfg<CT, 32, 64, BK>(gd, a, nz, s);
    case 5: return launch_cfg<CT, 64, 32, BK>(gd, a, nz, s);
    default: return launch_cfg<CT, 32, 32, BK>(gd, a, nz, s);
  }
}

std::string gemm_kernel_name(int ctype, const GemmDesc& gd) {
  static const int bm[] = {128, 64, 128, 64, 32, 64, 32};
  static const int bn[] = {128, 64, 64, 128, 64, 32, 32};
  const int t = gd.tile < 0 || gd.tile > 6 ? 6 : gd.tile;
  const int bk = ctype == 2 ? 32 : 16;
  return "ogemm_kernel<" + std::to_string(ctype) + ", " + std::to_string(bm[t]) + ", " + std::to_string(bn[t]) + ", " +
         std::to_string(bk) + ", " + (gd.a_mfast ? "true" : "false") + ", " + (gd.b_nfast ? "true" : "false") + ">";
}

hipError_t launch_gemm(int ctype, const GemmDesc& gd, const OpAddr& A, const OpAddr& B, const OpAddr& C,
                       const Epilogue& ep, int z0, int nz, int* flag, hipStream_t s) {
  KArgs a;
  a.A = kop(A, 2);
  a.B = kop(B, 2);
  a.C = kop(C, 2);
  a.has_d = ep.D.base != nullptr;
  a.D = a.has_d ? kop(ep.D, 2) : KOp{nullptr, nullptr, 0, 0, 0};
  a.flag = flag;
  a.a_om = gd.a_om;
  a.a_ok = gd.a_ok;
  a.b_ok = gd.b_ok;
  a.b_on = gd.b_on;
  a.c_om = gd.c_om;
  a.c_on = gd.c_on;
  a.alpha = ep.alpha;
  a.shift = ep.shift;
  a.M = gd.M;
  a.N = gd.N;
  a.K = gd.K;
  a.accum = ep.accum ? 1 : 0;
  a.d_const = ep.shift_const ? 1 : 0;
  for (int zz = 0; zz < nz; zz += 65535) {
    const int cnt = (nz - zz < 65535) ? nz - zz : 65535;
    a.z0 = z0 + zz;
    // chunk-local operands are indexed by z relative to the launch chunk
    KArgs b = a;
    if (b.A.mode == 3) b.A.base = (const char*)b.A.base + (int64_t)zz * b.A.bs * (ctype == 0 ? 8 : 4);
    if (b.B.mode == 3) b.B.base = (const char*)b.B.base + (int64_t)zz * b.B.bs * (ctype == 0 ? 8 : 4);
    if (b.C.mode == 3) b.C.base = (const char*)b.C.base + (int64_t)zz * b.C.bs * (ctype == 0 ? 8 : 4);
    hipError_t e;
    if (ctype == 0) e = launch_ct<0>(gd, b, cnt, s);
    else if (ctype == 1) e = launch_ct<1>(gd, b, cnt, s);
    else e = launch_ct<2>(gd, b, cnt, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------- batched dot
// out[z] = sum_i X_z[i] * Y_z[i], one workgroup per batch item, FP64 sum.
template <typename T>
__global__ __launch_bounds__(256) void bdot_kernel(const T* X, const int32_t* xtab, int64_t xs, const T* Y,
                                                   int64_t ys, int64_t n, int z0, double* out) {
  const int z = blockIdx.x;
  const T* x = X + (xtab ? (int64_t)xtab[z0 + z] : (int64_t)(z0 + z)) * xs;  // xtab validated by the caller
  const T* y = Y + (int64_t)z * ys;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc += (double)x[i] * (double)y[i];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[z0 + z] = red[0];
}

hipError_t launch_batched_dot(int ctype, const void* X, const int32_t* xtab, int64_t xstride, const void* Y,
                              int64_t ystride, int64_t n, int nz, int z0, double* out, hipStream_t s) {
  if (nz <= 0) return hipSuccess;
  if (ctype == 0)
    hipLaunchKernelGGL(bdot_kernel<double>, dim3(nz), dim3(256), 0, s, (const double*)X, xtab, xstride,
                       (const double*)Y, ystride, n, z0, out);
  else
    hipLaunchKernelGGL(bdot_kernel<float>, dim3(nz), dim3(256), 0, s, (const float*)X, xtab, xstride,
                       (const float*)Y, ystride, n, z0, out);
  return hipGetLastError();
}

}  // namespace ttn
