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

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "internal.h"

namespace ttn {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));
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
  int tiles, nz, xcd_remap;
  int* flag;  // flag[2] is raised when a batch table holds an out-of-range index
  const int32_t* gate;  // non-null: the launch does nothing when *gate == 0 (every thread reads the same word)
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

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2): linear id g runs on XCD g % 8.  With the XCD mapping on, the launch's
// (item, tile) list -- items in order, tiles of an item row by row -- is cut
// into 8 contiguous chunks and XCD x walks chunk x in order, so the
// workgroups in flight on one XCD work on one or two items and share their
// operand panels in that XCD's L2, and the XCDs get equal shares (measured
// on the 50-item 864 x 576 x 1008 stage: HBM reads 1.6 GB -> 0.46 GB per
// launch).  Off: a 2-D grid (tile, item).  Returns false for the padding
// workgroups of the last chunk.
__device__ __forceinline__ bool xcd_tile(const KArgs& g, int& z, int& tile) {
  if (g.xcd_remap) {
    const int total = g.tiles * g.nz;
    const int chunk = (total + 7) / 8;
    const int lin = (int)(blockIdx.x & 7) * chunk + (int)(blockIdx.x >> 3);
    if (lin >= total) return false;
    z = lin / g.tiles;
    tile = lin - z * g.tiles;
  } else {
    z = blockIdx.y;
    tile = blockIdx.x;
  }
  return true;
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
template <>
struct Types<3> {  // FP64 tensors, FP32 matrix cores
  typedef double T;
  typedef float L;
  typedef floatx4 Acc;
};

// k-offset tables up to this many entries are staged in LDS
#define KCAP 1536

// occupancy floor: 3 waves / SIMD for FP32 tiles, 2 for FP64 and bf16 tiles
template <int CT, int BM, int BN, int BK, bool AMF, bool BNF, bool CMF>
__global__ __launch_bounds__(256, (CT == 1) ? 3 : 2) void ogemm_kernel(KArgs g) {
  if (g.gate && *g.gate == 0) return;  // uniform, before any barrier
  typedef typename Types<CT>::T T;
  typedef typename Types<CT>::L L;
  typedef typename Types<CT>::Acc Acc;
  constexpr int EA = BM * BK / 256;
  constexpr int EB = BN * BK / 256;
  constexpr int WTM = BM / 2, WTN = BN / 2;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  // LDS layout per operand follows its fast global dimension, so that both the
  // staging stores and the MFMA fragment reads avoid bank conflicts:
  //  * m-fast (n-fast) operands: k-major slices [k][m + PM]; a fragment read
  //    takes 16 consecutive m of two adjacent k rows, PM puts those rows 16
  //    banks apart;
  //  * k-fast operands: m-major rows [m][k + PK]; PK makes the row stride 2
  //    modulo 32 banks so 16 rows x 2 k of a fragment read hit 32 banks.
  // bf16 always uses m-major rows (8 consecutive k per lane = one 16-byte read).
  constexpr bool A_KMAJOR = (CT != 2) && AMF;
  constexpr bool B_KMAJOR = (CT != 2) && BNF;
  constexpr int PM = (CT == 0) ? 2 : 16;
  constexpr int PK = (CT == 2) ? 8 : ((CT == 0) ? 1 : 2);
  constexpr int LA = A_KMAJOR ? BK * (BM + PM) : BM * (BK + PK);
  constexpr int LB = B_KMAJOR ? BK * (BN + PM) : BN * (BK + PK);
  __shared__ L As[2][LA];
  __shared__ L Bs[2][LB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  int z, tile;
  if (!xcd_tile(g, z, tile)) return;
  const int tmi = tile / g.tiles_n;
  const int tni = tile - tmi * g.tiles_n;
  const int m0 = tmi * BM, n0 = tni * BN;
  const int M = g.M, N = g.N, K = g.K;

  const T* __restrict__ A = (const T*)g.A.base + batch_off(g.A, z, g.z0, g.flag);
  const T* __restrict__ B = (const T*)g.B.base + batch_off(g.B, z, g.z0, g.flag);

  // ---- k-offset tables staged in LDS once (K <= KCAP), so the per-tile
  // address of an element costs an LDS read instead of a dependent global load
  // (dynamic LDS of 2 K ints, sized by the launch: a short-K stage keeps its
  // occupancy instead of reserving the table cap)
  extern __shared__ int sk_dyn[];
  int* sk_a = sk_dyn;
  int* sk_b = sk_dyn + K;
  const bool k_in_lds = K <= KCAP;
  if (k_in_lds) {
    for (int i = tid; i < K; i += 256) {
      sk_a[i] = g.a_ok[i];
      sk_b[i] = g.b_ok[i];
    }
  }

  // ---- fixed per-thread offsets (rows / columns owned by this thread);
  // invalid entries are clamped to offset 0 (always addressable) and masked
  int a_fix[AMF ? 1 : EA];
  int b_fix[BNF ? 1 : EB];
  bool a_ok_row[AMF ? 1 : EA], b_ok_col[BNF ? 1 : EB];
  if (AMF) {
    const int mg = m0 + tid % BM;
    a_ok_row[0] = mg < M;
    a_fix[0] = a_ok_row[0] ? g.a_om[mg] : 0;
  } else {
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int mg = m0 + tid / BK + i * (256 / BK);
      a_ok_row[i] = mg < M;
      a_fix[i] = a_ok_row[i] ? g.a_om[mg] : 0;
    }
  }
  if (BNF) {
    const int ng = n0 + tid % BN;
    b_ok_col[0] = ng < N;
    b_fix[0] = b_ok_col[0] ? g.b_on[ng] : 0;
  } else {
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int ng = n0 + tid / BK + i * (256 / BK);
      b_ok_col[i] = ng < N;
      b_fix[i] = b_ok_col[i] ? g.b_on[ng] : 0;
    }
  }
  // The epilogue's output offsets are loaded here, before the first barrier:
  // their latency overlaps the first slice's loads instead of following the
  // last slice (short-K stages are bound by that chain).
  T* __restrict__ C = (T*)g.C.base + batch_off(g.C, z, g.z0, g.flag);
  const T* __restrict__ Dp = g.has_d ? (const T*)g.D.base + batch_off(g.D, z, g.z0, g.flag) : nullptr;
  const double alpha = g.alpha ? g.alpha[g.z0 + z] : 1.0;
  const double sh = g.shift ? g.shift[g.z0 + z] : 0.0;
  constexpr int RI = CMF ? 1 : 4, CI = CMF ? 4 : 1;
  auto quad = [&](int i) { return (CT == 0) ? ((lane >> 4) + 4 * i) : (4 * (lane >> 4) + i); };
  auto ri = [](int i) { return CMF ? 0 : i; };
  auto ci = [](int i) { return CMF ? i : 0; };
  int cm[TM][RI], cn[TN][CI];
  bool rv[TM][RI], cv[TN][CI];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int mg = m0 + wm * WTM + a * 16 + (CMF ? (lane & 15) : quad(i));
      rv[a][i] = mg < M;
      cm[a][i] = rv[a][i] ? g.c_om[mg] : 0;
    }
#pragma unroll
  for (int b = 0; b < TN; ++b)
#pragma unroll
    for (int i = 0; i < CI; ++i) {
      const int ng = n0 + wn * WTN + b * 16 + (CMF ? quad(i) : (lane & 15));
      cv[b][i] = ng < N;
      cn[b][i] = cv[b][i] ? g.c_on[ng] : 0;
    }
  __syncthreads();

  // Next-slice loads are issued unconditionally from clamped, always valid
  // addresses (out-of-range k take the last table entry, out-of-range rows
  // offset 0; offsets are non-negative, so every sum stays inside the operand)
  // and the masks are applied only when the values are staged to LDS, after
  // the matrix-core work of the current slice: the loads of a slice are all in
  // flight together instead of each waiting for its own select.
  T ra[EA], rb[EB];
  bool kva[AMF ? EA : 1], kvb[BNF ? EB : 1];
  const int klast = K - 1;
  auto load = [&](int k0, auto lds_tab) {
    constexpr bool KL = decltype(lds_tab)::value;
    const int* __restrict__ ta = KL ? sk_a : g.a_ok;
    const int* __restrict__ tb = KL ? sk_b : g.b_ok;
    if (AMF) {
      int ko[EA];
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int kg = k0 + tid / BM + i * (256 / BM);
        kva[i] = kg < K;
        ko[i] = ta[kva[i] ? kg : klast];
      }
#pragma unroll
      for (int i = 0; i < EA; ++i) ra[i] = A[a_fix[0] + ko[i]];
    } else {
      const int kg = k0 + tid % BK;
      kva[0] = kg < K;
      const int ko = ta[kva[0] ? kg : klast];
#pragma unroll
      for (int i = 0; i < EA; ++i) ra[i] = A[a_fix[i] + ko];
    }
    if (BNF) {
      int ko[EB];
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int kg = k0 + tid / BN + i * (256 / BN);
        kvb[i] = kg < K;
        ko[i] = tb[kvb[i] ? kg : klast];
      }
#pragma unroll
      for (int i = 0; i < EB; ++i) rb[i] = B[b_fix[0] + ko[i]];
    } else {
      const int kg = k0 + tid % BK;
      kvb[0] = kg < K;
      const int ko = tb[kvb[0] ? kg : klast];
#pragma unroll
      for (int i = 0; i < EB; ++i) rb[i] = B[b_fix[i] + ko];
    }
  };
  auto aidx = [&](int m, int k) { return A_KMAJOR ? k * (BM + PM) + m : m * (BK + PK) + k; };
  auto bidx = [&](int n, int k) { return B_KMAJOR ? k * (BN + PM) + n : n * (BK + PK) + k; };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int ml = AMF ? tid % BM : tid / BK + i * (256 / BK);
      const int kl = AMF ? tid / BM + i * (256 / BM) : tid % BK;
      const bool ok = AMF ? (a_ok_row[0] && kva[i]) : (a_ok_row[i] && kva[0]);
      As[buf][aidx(ml, kl)] = ok ? (L)ra[i] : (L)0;
    }
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int nl = BNF ? tid % BN : tid / BK + i * (256 / BK);
      const int kl = BNF ? tid / BN + i * (256 / BN) : tid % BK;
      const bool ok = BNF ? (b_ok_col[0] && kvb[i]) : (b_ok_col[i] && kvb[0]);
      Bs[buf][bidx(nl, kl)] = ok ? (L)rb[i] : (L)0;
    }
  };

  Acc acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = Acc{0, 0, 0, 0};

  const int nk = (K + BK - 1) / BK;
  auto main_loop = [&](auto lds_tab) {
    if (nk <= 0) return;
    load(0, lds_tab);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) load((kt + 1) * BK, lds_tab);
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
            for (int b = 0; b < TN; ++b)
              acc[a][b] = CMF ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[b], af[a], acc[a][b], 0, 0, 0)
                              : __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
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
              const L x = CMF ? bfr[b] : af[a], y = CMF ? af[a] : bfr[b];
              if constexpr (CT == 0)
                acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[a][b], 0, 0, 0);
              else
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc[a][b], 0, 0, 0);
            }
        }
      }
      if (kt + 1 < nk) store(buf ^ 1);
      __syncthreads();
    }
  };
  // the table source is uniform over the launch: one specialised loop each
  if (k_in_lds)
    main_loop(std::true_type{});
  else
    main_loop(std::false_type{});

  // ---- epilogue: C = alpha (acc - shift * D) (+ C); output offsets loaded in
  // one batch, then the stores (masked rows / columns skipped).  Without CMF
  // a lane holds four rows of one column of each 16 x 16 block (lanes along
  // columns: coalesced when C's columns are its unit-stride direction); with
  // CMF the operands went into the matrix cores swapped, and a lane holds four
  // columns of one row (lanes along rows: coalesced when rows are unit-stride).
  const bool plain = !Dp && !g.d_const && !g.accum;
  if (plain) {
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < TN; ++b)
          if (rv[a][ri(i)] && cv[b][ci(i)]) C[cm[a][ri(i)] + cn[b][ci(i)]] = (T)(alpha * (double)acc[a][b][i]);
  } else {
    // per 16-row block: every read of the block first (masked rows and
    // columns read offset 0; a missing D reads C in its place and is replaced
    // by its constant afterwards), then its writes
    const T* __restrict__ ds = Dp ? Dp : (const T*)C;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      T dv[4][TN], cvv[4][TN];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const int o = cm[a][ri(i)] + cn[b][ci(i)];
          dv[i][b] = ds[o];
          cvv[i][b] = C[o];
        }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const double d = Dp ? (double)dv[i][b] : (g.d_const ? 1.0 : 0.0);
          const double c0 = g.accum ? (double)cvv[i][b] : 0.0;
          if (rv[a][ri(i)] && cv[b][ci(i)])
            C[cm[a][ri(i)] + cn[b][ci(i)]] = (T)(alpha * ((double)acc[a][b][i] - sh * d) + c0);
        }
    }
  }
}

// Unit-stride-k tile kernel, FP32 storage and arithmetic.  Both operands run
// contiguously along k (k offsets are exactly k, every row offset of A and
// column offset of B a multiple of 4 elements, 16-byte aligned bases,
// K % 4 == 0): the largest H_eff stages, where two intermediates meet over a
// (bond x operator bond) group.  Same 2 x 2 wave grid, XCD mapping and
// epilogue as ogemm_kernel, but every thread moves 16-byte runs of 4
// consecutive k: global loads are 16 bytes wide (8 lanes cover a 128-byte run
// of one row), an LDS row holds the slice's 8 runs of one row, written with
// one 16-byte store each, and a fragment read takes 4 consecutive k of one
// row in one 16-byte LDS read -- lane group q = l/16 supplies
// k = 16c + 4q + t to the t-th of the four MFMAs of 16-deep chunk c, for A
// and B alike, so every k is summed exactly once.  Run j of row r is stored
// at position j ^ (r & 7) of its LDS row: the 16 rows of a fragment read then
// hit distinct bank groups without padding (measured on the 864 x 576 x 1008
// stage: no bank-conflict cycles, 12% faster than a padded row).  BK = 32:
// one barrier per 32 k.
template <int BM, int BN, bool CMF, typename TS>
__global__ __launch_bounds__(256, 2) void ogemm_tn_kernel(KArgs g) {
  if (g.gate && *g.gate == 0) return;  // uniform, before any barrier
  constexpr int BK = 32, LR = BK / 4;  // LDS row: the slice's 8 runs of 4 k (float4), XOR-swizzled
  constexpr int EA = BM * BK / 4 / 256, EB = BN * BK / 4 / 256;
  constexpr int WTM = BM / 2, WTN = BN / 2;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  static_assert(EA >= 1 && EB >= 1 && TM >= 1 && TN >= 1, "tile too small");
  __shared__ floatx4 As[2][BM * LR];
  __shared__ floatx4 Bs[2][BN * LR];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  int z, tile;
  if (!xcd_tile(g, z, tile)) return;
  const int tmi = tile / g.tiles_n;
  const int tni = tile - tmi * g.tiles_n;
  const int m0 = tmi * BM, n0 = tni * BN;
  const int M = g.M, N = g.N, K = g.K;
  const TS* __restrict__ A = (const TS*)g.A.base + batch_off(g.A, z, g.z0, g.flag);
  const TS* __restrict__ B = (const TS*)g.B.base + batch_off(g.B, z, g.z0, g.flag);
  // a run of 4 consecutive k as loaded: FP32 storage one 16-byte load, FP64
  // storage two (converted to FP32 when staged in LDS)
  constexpr bool F64S = sizeof(TS) == 8;
  typedef typename std::conditional<F64S, doublex4, floatx4>::type Run;
  auto ld_run = [](const TS* p) -> Run {
    if constexpr (F64S) {
      const doublex2 lo = *(const doublex2*)p, hi = *(const doublex2*)(p + 2);
      return Run{lo[0], lo[1], hi[0], hi[1]};
    } else {
      return *(const floatx4*)p;
    }
  };
  auto to_f4 = [](const Run& r) -> floatx4 {
    if constexpr (F64S) return floatx4{(float)r[0], (float)r[1], (float)r[2], (float)r[3]};
    else return r;
  };

  // staging map: thread t moves k run jq = t % 8 of rows t / 8 + 32 i; rows
  // past M (N) read offset 0 (always addressable) and are zeroed in LDS
  const int jq = tid & 7, r0 = tid >> 3;
  int a_fix[EA], b_fix[EB];
  bool a_in[EA], b_in[EB];
#pragma unroll
  for (int i = 0; i < EA; ++i) {
    const int mg = m0 + r0 + 32 * i;
    a_in[i] = mg < M;
    a_fix[i] = a_in[i] ? g.a_om[mg] : 0;
  }
#pragma unroll
  for (int i = 0; i < EB; ++i) {
    const int ng = n0 + r0 + 32 * i;
    b_in[i] = ng < N;
    b_fix[i] = b_in[i] ? g.b_on[ng] : 0;
  }
  // Two register sets, so a slice's global loads are issued two slices
  // before they are staged: the wait at staging covers the matrix-core work
  // of two slices instead of one (the loop body is unrolled by two to keep
  // the sets in registers).  Tiles below 128 x 128 only.
  constexpr bool DEEP = BM * BN < 128 * 128;
  Run ra0[EA], rb0[EB], ra1[DEEP ? EA : 1], rb1[DEEP ? EB : 1];
  bool kv0 = false, kv1 = false;
  auto load = [&](Run* ra, Run* rb, bool& kv, int k0) {
    const int kg = k0 + 4 * jq;
    kv = kg < K;  // K % 4 == 0: a run lies wholly inside or outside [0, K)
    const int ko = kv ? kg : 0;
#pragma unroll
    for (int i = 0; i < EA; ++i) ra[i] = ld_run(A + a_fix[i] + ko);
#pragma unroll
    for (int i = 0; i < EB; ++i) rb[i] = ld_run(B + b_fix[i] + ko);
  };
  auto store = [&](const Run* ra, const Run* rb, bool kv, int buf) {
    const floatx4 z4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int r = r0 + 32 * i;
      As[buf][r * LR + (jq ^ (r & 7))] = (a_in[i] && kv) ? to_f4(ra[i]) : z4;
    }
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int r = r0 + 32 * i;
      Bs[buf][r * LR + (jq ^ (r & 7))] = (b_in[i] && kv) ? to_f4(rb[i]) : z4;
    }
  };

  floatx4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int nk = (K + BK - 1) / BK;
  const int fr = lane & 15, fq = lane >> 4;
  auto compute = [&](int buf) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      floatx4 fa[TM], fb[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        const int r = wm * WTM + a * 16 + fr;
        fa[a] = As[buf][r * LR + ((4 * c + fq) ^ (r & 7))];
      }
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int r = wn * WTN + b * 16 + fr;
        fb[b] = Bs[buf][r * LR + ((4 * c + fq) ^ (r & 7))];
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b)
            acc[a][b] = CMF ? __builtin_amdgcn_mfma_f32_16x16x4f32(fb[b][t], fa[a][t], acc[a][b], 0, 0, 0)
                            : __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a][t], fb[b][t], acc[a][b], 0, 0, 0);
    }
  };
  if constexpr (DEEP) {
    // slice s lives in register set s % 2 and LDS buffer s % 2
    if (nk > 0) {
      load(ra0, rb0, kv0, 0);
      if (nk > 1) load(ra1, rb1, kv1, BK);
      store(ra0, rb0, kv0, 0);
      __syncthreads();
    }
    for (int kt = 0; kt < nk; kt += 2) {
      if (kt + 2 < nk) load(ra0, rb0, kv0, (kt + 2) * BK);
      compute(0);
      if (kt + 1 < nk) store(ra1, rb1, kv1, 1);
      __syncthreads();
      if (kt + 1 >= nk) break;
      if (kt + 3 < nk) load(ra1, rb1, kv1, (kt + 3) * BK);
      compute(1);
      if (kt + 2 < nk) store(ra0, rb0, kv0, 0);
      __syncthreads();
    }
  } else {
    // one register set (the 128 x 128 tile has no registers for two)
    if (nk > 0) {
      load(ra0, rb0, kv0, 0);
      store(ra0, rb0, kv0, 0);
      __syncthreads();
    }
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) load(ra0, rb0, kv0, (kt + 1) * BK);
      compute(buf);
      if (kt + 1 < nk) store(ra0, rb0, kv0, buf ^ 1);
      __syncthreads();
    }
  }

  // ---- epilogue (as ogemm_kernel): C = alpha (acc - shift * D) (+ C)
  TS* __restrict__ C = (TS*)g.C.base + batch_off(g.C, z, g.z0, g.flag);
  const TS* __restrict__ Dp = g.has_d ? (const TS*)g.D.base + batch_off(g.D, z, g.z0, g.flag) : nullptr;
  const double alpha = g.alpha ? g.alpha[g.z0 + z] : 1.0;
  const double sh = g.shift ? g.shift[g.z0 + z] : 0.0;
  constexpr int RI = CMF ? 1 : 4, CI = CMF ? 4 : 1;
  auto quad = [&](int i) { return 4 * fq + i; };
  auto ri = [](int i) { return CMF ? 0 : i; };
  auto ci = [](int i) { return CMF ? i : 0; };
  int cm[TM][RI], cn[TN][CI];
  bool rv[TM][RI], cv[TN][CI];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int mg = m0 + wm * WTM + a * 16 + (CMF ? fr : quad(i));
      rv[a][i] = mg < M;
      cm[a][i] = rv[a][i] ? g.c_om[mg] : 0;
    }
#pragma unroll
  for (int b = 0; b < TN; ++b)
#pragma unroll
    for (int i = 0; i < CI; ++i) {
      const int ng = n0 + wn * WTN + b * 16 + (CMF ? quad(i) : fr);
      cv[b][i] = ng < N;
      cn[b][i] = cv[b][i] ? g.c_on[ng] : 0;
    }
  const bool plain = !Dp && !g.d_const && !g.accum;
  if (plain) {
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < TN; ++b)
          if (rv[a][ri(i)] && cv[b][ci(i)]) C[cm[a][ri(i)] + cn[b][ci(i)]] = (TS)(alpha * (double)acc[a][b][i]);
  } else {
    const TS* __restrict__ ds = Dp ? Dp : (const TS*)C;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      TS dv[4][TN], cvv[4][TN];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const int o = cm[a][ri(i)] + cn[b][ci(i)];
          dv[i][b] = ds[o];
          cvv[i][b] = C[o];
        }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const double d = Dp ? (double)dv[i][b] : (g.d_const ? 1.0 : 0.0);
          const double c0 = g.accum ? (double)cvv[i][b] : 0.0;
          if (rv[a][ri(i)] && cv[b][ci(i)])
            C[cm[a][ri(i)] + cn[b][ci(i)]] = (TS)(alpha * ((double)acc[a][b][i] - sh * d) + c0);
        }
    }
  }
}

// Wave-per-item variant for many tiny contractions (the identity-operator
// environments and local sums of a fitting sweep: thousands of (target,
// source) pairs with M, N of a few tens).  Each wave64 owns one batch item
// and walks its output in 16*TMW x 16*TNW tiles, feeding the matrix cores
// straight from global memory (no LDS staging, no workgroup barriers); the
// four waves of a workgroup take four consecutive items.
template <int CT, int TMW, int TNW>
__global__ __launch_bounds__(256) void ogemm_wave_kernel(KArgs g) {
  if (g.gate && *g.gate == 0) return;  // uniform, before any barrier
  typedef typename Types<CT == 2 ? 1 : CT>::T T;
  typedef typename Types<CT == 2 ? 1 : CT>::Acc Acc;
  const int lane = threadIdx.x & 63;
  const int z = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (z >= g.nz) return;  // wave-uniform; the kernel has no barriers
  const int M = g.M, N = g.N, K = g.K;
  const T* __restrict__ A = (const T*)g.A.base + batch_off(g.A, z, g.z0, g.flag);
  const T* __restrict__ B = (const T*)g.B.base + batch_off(g.B, z, g.z0, g.flag);
  T* __restrict__ C = (T*)g.C.base + batch_off(g.C, z, g.z0, g.flag);
  const T* __restrict__ Dp = g.has_d ? (const T*)g.D.base + batch_off(g.D, z, g.z0, g.flag) : nullptr;
  const double alpha = g.alpha ? g.alpha[g.z0 + z] : 1.0;
  const double sh = g.shift ? g.shift[g.z0 + z] : 0.0;
  const int l16 = lane & 15, lk = lane >> 4;
  for (int mt = 0; mt < M; mt += 16 * TMW) {
    int aoff[TMW];
    bool av_ok[TMW];
#pragma unroll
    for (int a = 0; a < TMW; ++a) {
      const int r = mt + a * 16 + l16;
      av_ok[a] = r < M;
      aoff[a] = av_ok[a] ? g.a_om[r] : 0;
    }
    for (int nt = 0; nt < N; nt += 16 * TNW) {
      int boff[TNW];
      bool bv_ok[TNW];
#pragma unroll
      for (int b = 0; b < TNW; ++b) {
        const int c = nt + b * 16 + l16;
        bv_ok[b] = c < N;
        boff[b] = bv_ok[b] ? g.b_on[c] : 0;
      }
      Acc acc[TMW][TNW];
#pragma unroll
      for (int a = 0; a < TMW; ++a)
#pragma unroll
        for (int b = 0; b < TNW; ++b) acc[a][b] = Acc{0, 0, 0, 0};
      for (int k0 = 0; k0 < K; k0 += 4) {
        const int kk = k0 + lk;
        const bool kv = kk < K;
        const int ak = kv ? g.a_ok[kk] : 0;
        const int bk = kv ? g.b_ok[kk] : 0;
        T af[TMW], bf[TNW];
#pragma unroll
        for (int a = 0; a < TMW; ++a) {
          const T v = A[aoff[a] + ak];
          af[a] = (kv && av_ok[a]) ? v : (T)0;
        }
#pragma unroll
        for (int b = 0; b < TNW; ++b) {
          const T v = B[bk + boff[b]];
          bf[b] = (kv && bv_ok[b]) ? v : (T)0;
        }
#pragma unroll
        for (int a = 0; a < TMW; ++a)
#pragma unroll
          for (int b = 0; b < TNW; ++b) {
            if constexpr (CT == 0)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
            else
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bf[b], acc[a][b], 0, 0, 0);
          }
      }
      // epilogue for this tile
#pragma unroll
      for (int a = 0; a < TMW; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = mt + a * 16 + ((CT == 0) ? (lk + 4 * i) : (4 * lk + i));
          const bool rok = row < M;
          const int cm = rok ? g.c_om[row] : 0;
#pragma unroll
          for (int b = 0; b < TNW; ++b) {
            const int col = nt + b * 16 + l16;
            if (!rok || col >= N) continue;
            const int o = cm + g.c_on[col];
            double v = (double)acc[a][b][i];
            if (Dp) v -= sh * (double)Dp[o];
            else if (g.d_const) v -= sh;
            v *= alpha;
            if (g.accum) v += (double)C[o];
            C[o] = (T)v;
          }
        }
    }
  }
}

// Split-K kernel for skinny products: M, N <= 32 with a long contraction whose
// operands both run contiguously along k (unit k stride, row offsets multiples
// of 4 elements: the identity-environment and fitting stages that reduce a
// whole node tensor to a bond x bond matrix).  One workgroup per batch item;
// its four waves take interleaved 16-wide k-chunks, every lane loads one
// 16-byte run of 4 consecutive k per operand row straight from global memory
// into f32 matrix-core operands (lane group q = l/16 supplies k = 4q + t to the
// t-th MFMA of a chunk, the same for A and B, so the sum over k is complete),
// the next chunk's loads are issued before the current chunk's MFMAs, and the
// four partial 32 x 32 accumulators are summed through LDS.  FP32 storage;
// the arithmetic is FP32 also for the bf16 compute type.
__global__ __launch_bounds__(256) void ogemm_splitk_kernel(KArgs g) {
  if (g.gate && *g.gate == 0) return;  // uniform, before any barrier
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int z = blockIdx.x;
  if (z >= g.nz) return;  // uniform per workgroup, before any barrier
  const int M = g.M, N = g.N, K = g.K;
  const float* __restrict__ A = (const float*)g.A.base + batch_off(g.A, z, g.z0, g.flag);
  const float* __restrict__ B = (const float*)g.B.base + batch_off(g.B, z, g.z0, g.flag);
  const int r = lane & 15, q = lane >> 4;
  // operand rows owned by this lane (rows past M / N read row 0 and are zeroed)
  const bool av0 = r < M, av1 = r + 16 < M, bv0 = r < N, bv1 = r + 16 < N;
  const float* a0p = A + (av0 ? g.a_om[r] : 0);
  const float* a1p = A + (av1 ? g.a_om[r + 16] : 0);
  const float* b0p = B + (bv0 ? g.b_on[r] : 0);
  const float* b1p = B + (bv1 ? g.b_on[r + 16] : 0);
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
  auto ld = [&](const float* p, bool row_ok, int k) -> floatx4 {
    // K % 4 == 0: a quad is either wholly inside [0, K) or wholly outside
    return (row_ok && k < K) ? *(const floatx4*)(p + k) : zero;
  };
  int c = wid;
  floatx4 x0 = ld(a0p, av0, c * 16 + 4 * q), x1 = ld(a1p, av1, c * 16 + 4 * q);
  floatx4 y0 = ld(b0p, bv0, c * 16 + 4 * q), y1 = ld(b1p, bv1, c * 16 + 4 * q);
  for (; c * 16 < K; c += 4) {
    const int kn = (c + 4) * 16 + 4 * q;
    const floatx4 nx0 = ld(a0p, av0, kn), nx1 = ld(a1p, av1, kn);
    const floatx4 ny0 = ld(b0p, bv0, kn), ny1 = ld(b1p, bv1, kn);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0[t], y0[t], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0[t], y1[t], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1[t], y0[t], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1[t], y1[t], acc[1][1], 0, 0, 0);
    }
    x0 = nx0;
    x1 = nx1;
    y0 = ny0;
    y1 = ny1;
  }
  // partial sums of the four waves: red[w][block][i][lane]
  __shared__ float red[4][4][4][64];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) red[wid][2 * i + j][e][lane] = acc[i][j][e];
  __syncthreads();
  // thread -> (block = wid, lane): its 4 output elements
  const int blk = wid, bi = blk >> 1, bj = blk & 1;
  float* __restrict__ C = (float*)g.C.base + batch_off(g.C, z, g.z0, g.flag);
  const float* __restrict__ Dp = g.has_d ? (const float*)g.D.base + batch_off(g.D, z, g.z0, g.flag) : nullptr;
  const double alpha = g.alpha ? g.alpha[g.z0 + z] : 1.0;
  const double sh = g.shift ? g.shift[g.z0 + z] : 0.0;
  const int col = bj * 16 + (lane & 15);
  const bool cok = col < N;
  const int cn = cok ? g.c_on[col] : 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int row = bi * 16 + 4 * (lane >> 4) + e;
    const float v = red[0][blk][e][lane] + red[1][blk][e][lane] + red[2][blk][e][lane] + red[3][blk][e][lane];
    if (row < M && cok) {
      const int o = g.c_om[row] + cn;
      const double dv = Dp ? (double)Dp[o] : (g.d_const ? 1.0 : 0.0);
      const double cv = g.accum ? (double)C[o] : 0.0;
      C[o] = (float)(alpha * ((double)v - sh * dv) + cv);
    }
  }
}

// Narrow kernel: tall M, N <= 32 and a short unit-stride contraction
// (K <= 32), both operands contiguous along k (the first stages of identity
// environments: one bond of a node tensor contracted with a bond x bond
// matrix).  One workgroup per batch item; every lane keeps its B fragments
// (N <= 32 columns x K <= 32) in registers for the whole item, the four waves
// walk the M rows in 16-row blocks, loading each lane's A row as 16-byte runs
// of k (next block prefetched before the current block's MFMAs), and write C
// through the output offset tables.  FP32 arithmetic.
template <bool CMF>
__global__ __launch_bounds__(256) void ogemm_narrow_kernel(KArgs g) {
  if (g.gate && *g.gate == 0) return;  // uniform
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int z = blockIdx.x;
  if (z >= g.nz) return;  // no barriers below: waves may leave independently
  const int M = g.M, N = g.N, K = g.K;
  const float* __restrict__ A = (const float*)g.A.base + batch_off(g.A, z, g.z0, g.flag);
  const float* __restrict__ B = (const float*)g.B.base + batch_off(g.B, z, g.z0, g.flag);
  float* __restrict__ C = (float*)g.C.base + batch_off(g.C, z, g.z0, g.flag);
  const float* __restrict__ Dp = g.has_d ? (const float*)g.D.base + batch_off(g.D, z, g.z0, g.flag) : nullptr;
  const double alpha = g.alpha ? g.alpha[g.z0 + z] : 1.0;
  const double sh = g.shift ? g.shift[g.z0 + z] : 0.0;
  const int r = lane & 15, q = lane >> 4;
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
  // k quads of this lane (K % 4 == 0: a quad lies wholly inside or outside [0, K));
  // quads past K read quad 0 and are zeroed before use
  const bool kq[2] = {4 * q < K, 16 + 4 * q < K};
  const int kof[2] = {kq[0] ? 4 * q : 0, kq[1] ? 16 + 4 * q : 0};
  // B fragments: column r (+16), k = 16 h + 4 q .. +3
  floatx4 bq[2][2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int col = nb * 16 + r;
    const bool ok = col < N;
    const float* bp = B + (ok ? g.b_on[col] : 0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const floatx4 v = *(const floatx4*)(bp + kof[h]);
      bq[nb][h] = (ok && kq[h]) ? v : zero;
    }
  }
  // Output placement of acc[nb][e] for the 16-row block mb: without CMF row
  // 16 mb + 4 q + e, column 16 nb + r (lanes along columns); with CMF the
  // matrix-core operands are swapped and it is row 16 mb + r, column
  // 16 nb + 4 q + e (lanes along rows, for outputs whose rows are unit-stride).
  constexpr int RI = CMF ? 1 : 4, CI = CMF ? 4 : 1;
  int cn[2][CI];
  bool cok[2][CI];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int i = 0; i < CI; ++i) {
      const int col = nb * 16 + (CMF ? 4 * q + i : r);
      cok[nb][i] = col < N;
      cn[nb][i] = cok[nb][i] ? g.c_on[col] : 0;
    }
  auto ri = [](int e) { return CMF ? 0 : e; };
  auto ci = [](int e) { return CMF ? e : 0; };
  auto out_row = [&](int blk, int i) { return blk * 16 + (CMF ? r : 4 * q + i); };
  const int nmb = (M + 15) / 16;
  int mb = wid;
  if (mb >= nmb) return;
  // Software pipeline over this wave's 16-row blocks mb, mb + 4, ...: while the
  // current block is multiplied and written, the next block's A rows and output
  // row offsets are in flight, and the row offset of the block after that.
  // Rows past M are clamped to row 0 (read, never written).
  auto clamp_row = [&](int row) { return row < M ? row : 0; };
  int ao_next = g.a_om[clamp_row((mb + 4) * 16 + r)];
  const float* ap = A + g.a_om[clamp_row(mb * 16 + r)];
  floatx4 aq[2] = {*(const floatx4*)(ap + kof[0]), *(const floatx4*)(ap + kof[1])};
  int cm[RI];
#pragma unroll
  for (int i = 0; i < RI; ++i) cm[i] = g.c_om[clamp_row(out_row(mb, i))];
  const bool plain = !Dp && !g.d_const && !g.accum;
  for (; mb < nmb; mb += 4) {
    // issue: the offset two blocks ahead first (the oldest load of this round
    // is then the one the next round waits on), then the next block's data
    const int ao_after = g.a_om[clamp_row((mb + 8) * 16 + r)];
    const float* apn = A + ao_next;
    floatx4 an[2] = {*(const floatx4*)(apn + kof[0]), *(const floatx4*)(apn + kof[1])};
    int cmn[RI];
#pragma unroll
    for (int i = 0; i < RI; ++i) cmn[i] = g.c_om[clamp_row(out_row(mb + 4, i))];
    floatx4 acc[2] = {zero, zero};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (16 * h >= K) break;
      const floatx4 a = kq[h] ? aq[h] : zero;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if constexpr (CMF) {
          acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(bq[0][h][t], a[t], acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(bq[1][h][t], a[t], acc[1], 0, 0, 0);
        } else {
          acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], bq[0][h][t], acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], bq[1][h][t], acc[1], 0, 0, 0);
        }
      }
    }
    bool rok[RI];
#pragma unroll
    for (int i = 0; i < RI; ++i) rok[i] = out_row(mb, i) < M;
    if (plain) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          if (rok[ri(e)] && cok[nb][ci(e)]) C[cm[ri(e)] + cn[nb][ci(e)]] = (float)(alpha * (double)acc[nb][e]);
    } else {
      // all reads of the epilogue first (unconditional: a missing D reads C
      // in its place and is replaced by its constant afterwards), then the writes
      const float* __restrict__ ds = Dp ? Dp : C;
      const float dc = g.d_const ? 1.f : 0.f;
      float dv[4][2], cv[4][2];
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const int o = cm[ri(e)] + cn[nb][ci(e)];
          dv[e][nb] = ds[o];
          cv[e][nb] = C[o];
        }
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const double d = Dp ? (double)dv[e][nb] : (double)dc;
          const double c0 = g.accum ? (double)cv[e][nb] : 0.0;
          if (rok[ri(e)] && cok[nb][ci(e)])
            C[cm[ri(e)] + cn[nb][ci(e)]] = (float)(alpha * ((double)acc[nb][e] - sh * d) + c0);
        }
    }
    aq[0] = an[0];
    aq[1] = an[1];
#pragma unroll
    for (int i = 0; i < RI; ++i) cm[i] = cmn[i];
    ao_next = ao_after;
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

static int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return v ? atoi(v) : dflt;
}

template <int CT, int BM, int BN, int BK>
static hipError_t launch_cfg(const GemmDesc& gd, KArgs& a, int nz, hipStream_t s) {
  const int tm = (gd.M + BM - 1) / BM, tn = (gd.N + BN - 1) / BN;
  a.tiles_n = tn;
  a.tiles = tm * tn;
  a.nz = nz;
  static const int remap_min = env_int("TTN_XCD_REMAP_MIN", 16);  // workgroups: below that one XCD round
  a.xcd_remap = (int64_t)a.tiles * nz >= remap_min ? 1 : 0;
  dim3 grid = a.xcd_remap ? dim3((unsigned)(((int64_t)a.tiles * nz + 7) / 8 * 8), 1) : dim3(tm * tn, nz);
  const size_t kt = gd.K <= KCAP ? (size_t)2 * gd.K * sizeof(int) : 0;  // k-offset tables in LDS
  if (gd.c_mfast) {
    if (gd.a_mfast && gd.b_nfast) hipLaunchKernelGGL((ogemm_kernel<CT, BM, BN, BK, true, true, true>), grid, dim3(256), kt, s, a);
    else if (gd.a_mfast) hipLaunchKernelGGL((ogemm_kernel<CT, BM, BN, BK, true, false, true>), grid, dim3(256), kt, s, a);
    else if (gd.b_nfast) hipLaunchKernelGGL((ogemm_kernel<CT, BM, BN, BK, false, true, true>), grid, dim3(256), kt, s, a);
    else hipLaunchKernelGGL((ogemm_kernel<CT, BM, BN, BK, false, false, true>), grid, dim3(256), kt, s, a);
  } else {
    if (gd.a_mfast && gd.b_nfast) hipLaunchKernelGGL((ogemm_kernel<CT, BM, BN, BK, true, true, false>), grid, dim3(256), kt, s, a);
    else if (gd.a_mfast) hipLaunchKernelGGL((ogemm_kernel<CT, BM, BN, BK, true, false, false>), grid, dim3(256), kt, s, a);
    else if (gd.b_nfast) hipLaunchKernelGGL((ogemm_kernel<CT, BM, BN, BK, false, true, false>), grid, dim3(256), kt, s, a);
    else hipLaunchKernelGGL((ogemm_kernel<CT, BM, BN, BK, false, false, false>), grid, dim3(256), kt, s, a);
  }
  return hipGetLastError();
}

template <int CT, int BK>
static hipError_t launch_tile(const GemmDesc& gd, KArgs& a, int nz, hipStream_t s) {
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

// unit-stride-k tiles (ids 10..16) and the general tile each falls back to
// when a launch's operands are not 16-byte aligned
template <int BM, int BN, typename TS>
static hipError_t launch_tn(const GemmDesc& gd, KArgs& a, int nz, hipStream_t s) {
  const int tm = (gd.M + BM - 1) / BM, tn = (gd.N + BN - 1) / BN;
  a.tiles_n = tn;
  a.tiles = tm * tn;
  a.nz = nz;
  static const int remap_min = env_int("TTN_XCD_REMAP_MIN", 16);  // workgroups: below that one XCD round
  a.xcd_remap = (int64_t)a.tiles * nz >= remap_min ? 1 : 0;
  dim3 grid = a.xcd_remap ? dim3((unsigned)(((int64_t)a.tiles * nz + 7) / 8 * 8), 1) : dim3(tm * tn, nz);
  if (gd.c_mfast) hipLaunchKernelGGL((ogemm_tn_kernel<BM, BN, true, TS>), grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((ogemm_tn_kernel<BM, BN, false, TS>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename TS>
static hipError_t launch_tn_tile(const GemmDesc& gd, KArgs& a, int nz, hipStream_t s) {
  switch (gd.tile) {
    case 10: return launch_tn<128, 128, TS>(gd, a, nz, s);
    case 11: return launch_tn<128, 64, TS>(gd, a, nz, s);
    case 12: return launch_tn<64, 128, TS>(gd, a, nz, s);
    case 13: return launch_tn<64, 64, TS>(gd, a, nz, s);
    case 14: return launch_tn<96, 96, TS>(gd, a, nz, s);
    case 15: return launch_tn<64, 32, TS>(gd, a, nz, s);
    default: return launch_tn<128, 32, TS>(gd, a, nz, s);
  }
}

static const int kTnBM[] = {128, 128, 64, 64, 96, 64, 128};
static const int kTnBN[] = {128, 64, 128, 64, 96, 32, 32};
static const int kTnFallback[] = {0, 2, 3, 1, 0, 5, 2};

// k-slice depth: 16 for FP32 and FP64 (measured on the hot-path shapes: a
// deeper FP32 slice costs occupancy and never paid), 32 for bf16 (one MFMA).
static int pick_bk(int ctype) { return ctype == 2 ? 32 : 16; }

template <int CT>
static hipError_t launch_wave(const GemmDesc& gd, KArgs& a, int nz, hipStream_t s) {
  a.nz = nz;
  a.xcd_remap = 0;
  dim3 grid((unsigned)((nz + 3) / 4));
  constexpr int C2 = (CT == 2) ? 1 : CT;  // tiny stages of a bf16 contraction run on FP32 matrix cores
  if (gd.M <= 16 && gd.N <= 16) hipLaunchKernelGGL((ogemm_wave_kernel<C2, 1, 1>), grid, dim3(256), 0, s, a);
  else if (gd.M <= 16) hipLaunchKernelGGL((ogemm_wave_kernel<C2, 1, 2>), grid, dim3(256), 0, s, a);
  else if (gd.N <= 16) hipLaunchKernelGGL((ogemm_wave_kernel<C2, 2, 1>), grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((ogemm_wave_kernel<C2, 2, 2>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

static bool aligned16(const KOp& o) {
  return ((uintptr_t)o.base % 16) == 0 && (o.mode == 0 || o.bs % 4 == 0);
}

template <int CT>
static hipError_t launch_ct(const GemmDesc& gd, KArgs& a, int nz, hipStream_t s) {
  if (gd.tile == 8) {
    if (CT != 0 && splitk_eligible(gd, CT) && aligned16(a.A) && aligned16(a.B)) {
      a.nz = nz;
      a.xcd_remap = 0;
      hipLaunchKernelGGL(ogemm_splitk_kernel, dim3((unsigned)nz), dim3(256), 0, s, a);
      return hipGetLastError();
    }
    GemmDesc g2 = gd;
    g2.tile = 6;  // operands not 16-byte aligned: the general 32 x 32 tile
    return launch_ct<CT>(g2, a, nz, s);
  }
  if (gd.tile == 9) {
    if (CT != 0 && narrow_eligible(gd, CT) && aligned16(a.A) && aligned16(a.B)) {
      a.nz = nz;
      a.xcd_remap = 0;
      if (gd.c_mfast) hipLaunchKernelGGL(ogemm_narrow_kernel<true>, dim3((unsigned)nz), dim3(256), 0, s, a);
      else hipLaunchKernelGGL(ogemm_narrow_kernel<false>, dim3((unsigned)nz), dim3(256), 0, s, a);
      return hipGetLastError();
    }
    GemmDesc g2 = gd;
    g2.tile = 5;  // operands not 16-byte aligned: the general 64 x 32 tile
    return launch_ct<CT>(g2, a, nz, s);
  }
  if (gd.tile >= 10 && gd.tile <= 16) {
    if constexpr (CT == 1 || CT == 3) {
      if (tn_eligible(gd, CT) && aligned16(a.A) && aligned16(a.B))
        return launch_tn_tile<typename std::conditional<CT == 3, double, float>::type>(gd, a, nz, s);
    }
    GemmDesc g2 = gd;
    g2.tile = kTnFallback[gd.tile - 10];
    return launch_ct<CT>(g2, a, nz, s);
  }
  if (gd.tile == 7) {
    if constexpr (CT == 3) {
      GemmDesc g2 = gd;
      g2.tile = 6;  // no wave-per-item variant for FP64 storage with FP32 arithmetic
      return launch_tile<CT, 16>(g2, a, nz, s);
    } else {
      return launch_wave<CT>(gd, a, nz, s);
    }
  }
  return launch_tile<CT, (CT == 2) ? 32 : 16>(gd, a, nz, s);
}


std::string gemm_kernel_name(int ctype, const GemmDesc& gd) {
  static const int bm[] = {128, 64, 128, 64, 32, 64, 32};
  static const int bn[] = {128, 64, 64, 128, 64, 32, 32};
  if (gd.tile == 8) return "ogemm_splitk_kernel";
  if (gd.tile >= 10 && gd.tile <= 16) {
    if (tn_eligible(gd, ctype))
      return "ogemm_tn_kernel<" + std::to_string(kTnBM[gd.tile - 10]) + ", " + std::to_string(kTnBN[gd.tile - 10]) +
             ", " + (gd.c_mfast ? "true" : "false") + (ctype == 3 ? ", double>" : ">");
    GemmDesc g2 = gd;
    g2.tile = kTnFallback[gd.tile - 10];
    return gemm_kernel_name(ctype, g2);
  }
  if (gd.tile == 9) return std::string("ogemm_narrow_kernel<") + (gd.c_mfast ? "true" : "false") + ">";
  if (gd.tile == 7) {
    const int tmw = gd.M <= 16 ? 1 : 2, tnw = gd.N <= 16 ? 1 : 2;
    return "ogemm_wave_kernel<" + std::to_string(ctype == 2 ? 1 : ctype) + ", " + std::to_string(tmw) + ", " +
           std::to_string(tnw) + ">";
  }
  const int t = gd.tile < 0 || gd.tile > 6 ? 6 : gd.tile;
  const int bk = pick_bk(ctype);
  return "ogemm_kernel<" + std::to_string(ctype) + ", " + std::to_string(bm[t]) + ", " + std::to_string(bn[t]) + ", " +
         std::to_string(bk) + ", " + (gd.a_mfast ? "true" : "false") + ", " + (gd.b_nfast ? "true" : "false") + ", " +
         (gd.c_mfast ? "true" : "false") + ">";
}

hipError_t launch_gemm(int ctype, const GemmDesc& gd, const OpAddr& A, const OpAddr& B, const OpAddr& C,
                       const Epilogue& ep, int z0, int nz, int* flag, hipStream_t s, const int32_t* gate) {
  KArgs a;
  a.A = kop(A, 2);
  a.B = kop(B, 2);
  a.C = kop(C, 2);
  a.has_d = ep.D.base != nullptr;
  a.D = a.has_d ? kop(ep.D, 2) : KOp{nullptr, nullptr, 0, 0, 0};
  a.flag = flag;
  a.gate = gate;
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
    if (b.A.mode == 3) b.A.base = (const char*)b.A.base + (int64_t)zz * b.A.bs * ((ctype == 0 || ctype == 3) ? 8 : 4);
    if (b.B.mode == 3) b.B.base = (const char*)b.B.base + (int64_t)zz * b.B.bs * ((ctype == 0 || ctype == 3) ? 8 : 4);
    if (b.C.mode == 3) b.C.base = (const char*)b.C.base + (int64_t)zz * b.C.bs * ((ctype == 0 || ctype == 3) ? 8 : 4);
    hipError_t e;
    if (ctype == 0) e = launch_ct<0>(gd, b, cnt, s);
    else if (ctype == 1) e = launch_ct<1>(gd, b, cnt, s);
    else if (ctype == 2) e = launch_ct<2>(gd, b, cnt, s);
    else e = launch_ct<3>(gd, b, cnt, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------- relayout
// dst[k * M + m] = src[om[m] + ok[k]]: a shared operand copied into the
// row-fast order its GEMM reads (consecutive threads write consecutive m).
template <typename T>
__global__ __launch_bounds__(256) void relayout_kernel(const T* __restrict__ src, const int32_t* __restrict__ om,
                                                       const int32_t* __restrict__ ok, int M, int K,
                                                       T* __restrict__ dst, const int32_t* gate) {
  if (gate && *gate == 0) return;
  const int64_t total = (int64_t)M * K;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int k = (int)(i / M), m = (int)(i - (int64_t)k * M);
    dst[i] = src[om[m] + ok[k]];
  }
}

hipError_t launch_relayout(int ctype, const void* src, const int32_t* om, const int32_t* ok, int M, int K, void* dst,
                           hipStream_t s, const int32_t* gate) {
  const int64_t total = (int64_t)M * K;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  if (total <= 0) return hipSuccess;
  if (ctype == 0 || ctype == 3)
    hipLaunchKernelGGL(relayout_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double*)src, om, ok, M, K,
                       (double*)dst, gate);
  else
    hipLaunchKernelGGL(relayout_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float*)src, om, ok, M, K,
                       (float*)dst, gate);
  return hipGetLastError();
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
