// Fused identity-operator environment update for a node with three virtual
// legs and no physical leg (the internal nodes of a binary tree whose modes sit
// on the leaves), FP32 storage and FP32 matrix cores.
//
// The environment toward leg o of node u (Sec. II.B, the overlap
// environments of the Gram step) is, for one (bra, ket) pair,
//   E_o[x_o][y_o] = sum bra[x_o, x_p, x_q] E_p[x_p][y_p] E_q[x_q][y_q] ket[y_o, y_p, y_q],
// with p, q the other two legs and E_p, E_q the incoming environments
// (rows: bra bond, columns: ket bond).  One workgroup per pair:
//   1. the ket tensor is staged in LDS as rows K_y = ket[y, :, :] (Dp x Dq);
//   2. K_y is replaced in place by V_y = E_p K_y E_q^T for every y, as two
//      wide matrix-core products (E_p times all rows of the ket, then the
//      stacked result times E_q^T) split into 16-wide blocks over the waves;
//   3. E_o = Bra V^T with Bra = bra viewed as Do x (Dp Dq): the Dp Dq
//      contraction is split over the four waves, partial 32 x 32 blocks are
//      summed through LDS and written.
// The staged contraction path computes the same three products through HBM
// intermediates; here they never leave the workgroup.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ttn {

typedef float floatx4 __attribute__((ext_vector_type(4)));

#define IE_LD 33  // row stride of the 32 x 32 LDS tiles (one pad word)

__device__ __forceinline__ void ie_products(float* sV, const float (&ea)[8][2], const float (&eb)[8][2], int Do,
                                            int Dp, int Dq, int PQS);

// Shared first phase: the tensor X (legs 0, 1, 2 of dims dm0..dm2 in memory
// order, no physical leg) is staged in LDS as rows K_y = X[y over leg lo, :, :]
// (Dp x Dq, row stride PQS), E_p and E_q zero-padded to 32 x 32, and the rows
// are replaced by V_y = E_p K_y E_q^T (two MFMA products over all y at once,
// 16-wide blocks dealt to the waves).  Ends with a workgroup barrier; sT is
// not used here.
__device__ __forceinline__ void ie_stage_v(const float* __restrict__ ket, const float* __restrict__ Ep,
                                           const float* __restrict__ Eq, float* sV, float* sEp, float* sEq,
                                           float* sT, int dm0, int dm1, int dm2, int lo, int lp, int lq, int Do,
                                           int Dp, int Dq, int PQS) {
  (void)sT;
  const int tid = threadIdx.x, lane = tid & 63;
  const int r = lane & 15, gq = lane >> 4;
  const int D1 = dm1, D2 = dm2, D1D2 = D1 * D2;
  const int n3 = dm0 * D1D2;
  // LDS strides of the three tensor legs, and the thread's tensor index
  // advanced by 256 elements per round without divisions
  int ls[3];
  ls[lo] = PQS;
  ls[lp] = Dq;
  ls[lq] = 1;
  const int c0 = 256 / D1D2, c1 = (256 - c0 * D1D2) / D2, c2 = 256 - c0 * D1D2 - c1 * D2;
  int i0 = tid / D1D2, i1 = (tid - i0 * D1D2) / D2, i2 = tid - i0 * D1D2 - i1 * D2;
  // eight loads in flight per thread, then their stores
  for (int e0 = tid; e0 < n3; e0 += 256 * 8) {
    float kv8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = e0 + 256 * j;
      kv8[j] = ket[e < n3 ? e : 0];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = e0 + 256 * j;
      if (e < n3) sV[i0 * ls[0] + i1 * ls[1] + i2 * ls[2]] = kv8[j];
      i2 += c2;
      if (i2 >= D2) {
        i2 -= D2;
        ++i1;
      }
      i1 += c1;
      if (i1 >= D1) {
        i1 -= D1;
        ++i0;
      }
      i0 += c0;
    }
  }
  for (int e = tid; e < 32 * 32; e += 256) {
    const int a = e >> 5, b = e & 31;
    sEp[a * IE_LD + b] = (a < Dp && b < Dp) ? Ep[a * Dp + b] : 0.f;
    sEq[a * IE_LD + b] = (a < Dq && b < Dq) ? Eq[a * Dq + b] : 0.f;
  }
  __syncthreads();
  float ea[8][2], eb[8][2];  // E_p and E_q^T fragments of this lane (zero-padded)
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      ea[s][mi] = sEp[(16 * mi + r) * IE_LD + 4 * s + gq];
      eb[s][mi] = sEq[(16 * mi + r) * IE_LD + 4 * s + gq];
    }
  ie_products(sV, ea, eb, Do, Dp, Dq, PQS);
}

// The two wide products of the shared phase on the rows K_y staged in sV,
// with this lane's zero-padded fragments ea[s][mi] = E_p[16 mi + r][4 s + gq]
// and eb[s][ni] = E_q[16 ni + r][4 s + gq] (r = lane % 16, gq = lane / 16):
// K_y becomes V_y = E_p K_y E_q^T in place.  The caller has staged the rows
// behind a workgroup barrier; ends with a barrier before the readers of V.
__device__ __forceinline__ void ie_products(float* sV, const float (&ea)[8][2], const float (&eb)[8][2], int Do,
                                            int Dp, int Dq, int PQS) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int r = lane & 15, gq = lane >> 4;
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
  const int sp_steps = (Dp + 3) >> 2, sq_steps = (Dq + 3) >> 2;
  const int mta = (Dp + 15) >> 4, ntb = (Dq + 15) >> 4;
  const int ncol = Do * Dq, nrow = Do * Dp;
  {
    for (int cb = wid; cb * 16 < ncol; cb += 4) {
      const int c = 16 * cb + r;
      const bool cv = c < ncol;
      const int y = cv ? c / Dq : 0, yq = cv ? c - y * Dq : 0;
      float* col = sV + y * PQS + yq;  // element y_p of column c at col[y_p * Dq]
      floatx4 acc[2] = {zero, zero};
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        if (s >= sp_steps) break;
        const int k = 4 * s + gq;
        const float b = (cv && k < Dp) ? col[k * Dq] : 0.f;
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
          if (mi < mta) acc[mi] = __builtin_amdgcn_mfma_f32_16x16x4f32(ea[s][mi], b, acc[mi], 0, 0, 0);
      }
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int xp = 16 * mi + 4 * gq + i;
          if (mi < mta && cv && xp < Dp) col[xp * Dq] = acc[mi][i];
        }
    }
  }
  __syncthreads();
  {
    for (int rb = wid; rb * 16 < nrow; rb += 4) {
      const int R = 16 * rb + r;
      const bool rv = R < nrow;
      const int y = rv ? R / Dp : 0, xp = rv ? R - y * Dp : 0;
      const float* row = sV + y * PQS + xp * Dq;
      floatx4 acc[2] = {zero, zero};
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        if (s >= sq_steps) break;
        const int k = 4 * s + gq;
        const float a = (rv && k < Dq) ? row[k] : 0.f;
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          if (ni < ntb) acc[ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, eb[s][ni], acc[ni], 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int R2 = 16 * rb + 4 * gq + i;
        if (R2 < nrow) {
          const int y2 = R2 / Dp, xp2 = R2 - y2 * Dp;
          float* orow = sV + y2 * PQS + xp2 * Dq;
#pragma unroll
          for (int ni = 0; ni < 2; ++ni) {
            const int xq = 16 * ni + r;
            if (ni < ntb && xq < Dq) orow[xq] = acc[ni][i];
          }
        }
      }
    }
  }
  __syncthreads();

}


// ---- compile-time shapes: every global load of an item issued up front
//
// The load phase of one item is a single memory latency: the tensor as
// 16-byte runs (C2 % 4 == 0, rows 16-byte aligned; the launcher checks),
// the environment fragments and, in the environment kernel, the bra
// fragments of the last product are all in flight before the first of them
// is used, and only the tensor is waited for before the LDS products.

template <int N3>
constexpr int ie_pt = (N3 / 4 + 255) / 256;  // 16-byte loads per thread

// kv[j] = X[4 (tid + 256 j) .. +3] (the tail of the last round re-reads
// element 0 and is never stored)
template <int N3>
__device__ __forceinline__ void ie_load_x(const float* __restrict__ X, floatx4 (&kv)[ie_pt<N3>]) {
  constexpr int NV = N3 / 4;
#pragma unroll
  for (int j = 0; j < ie_pt<N3>; ++j) {
    const int e4 = threadIdx.x + 256 * j;
    kv[j] = *(const floatx4*)(X + 4 * (e4 < NV ? e4 : 0));
  }
}

// element (i0, i1, i2) of the C0 x C1 x C2 tensor to sV[i0 ls0 + i1 ls1 + i2 ls2]
template <int C0, int C1, int C2>
__device__ __forceinline__ void ie_store_x(const floatx4 (&kv)[ie_pt<C0 * C1 * C2>], float* sV, int ls0, int ls1,
                                           int ls2) {
  constexpr int NV = C0 * C1 * C2 / 4;
#pragma unroll
  for (int j = 0; j < ie_pt<C0 * C1 * C2>; ++j) {
    const int e4 = threadIdx.x + 256 * j;
    if (e4 < NV) {
      const int e = 4 * e4;
      const int i0 = e / (C1 * C2), rem = e - i0 * (C1 * C2);
      const int i1 = rem / C2, i2 = rem - i1 * C2;
      float* d = sV + i0 * ls0 + i1 * ls1 + i2 * ls2;
#pragma unroll
      for (int t = 0; t < 4; ++t) d[t * ls2] = kv[j][t];
    }
  }
}

// f[s][i] = E[16 i + r][4 s + gq] of the DE x DE environment, zero outside
template <int DE>
__device__ __forceinline__ void ie_efrag(const float* __restrict__ E, float (&f)[8][2]) {
  const int lane = threadIdx.x & 63, r = lane & 15, gq = lane >> 4;
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = 16 * i + r, col = 4 * s + gq;
      f[s][i] = (4 * s < DE && 16 * i < DE && row < DE && col < DE) ? E[row * DE + col] : 0.f;
    }
}


// ie_products with compile-time dims (D_p, D_q multiples of 4, D_o D_p and
// D_o D_q multiples of 16): the operands of a wave's next 16-wide block are
// read from LDS before the MFMAs of the current one, so LDS latency hides
// under the matrix pipe; rows and columns past the dims are never stored, so
// the padded lanes read any in-range element instead of being masked.
template <int DO, int DP, int DQ>
__device__ __forceinline__ void ie_products_ct(float* sV, const float (&ea)[8][2], const float (&eb)[8][2], int PQS) {
  static_assert(DP % 4 == 0 && DQ % 4 == 0 && (DO * DP) % 16 == 0 && (DO * DQ) % 16 == 0 && DP <= 32 && DQ <= 32,
                "compile-time product shapes");
  constexpr int SP = DP / 4, SQ = DQ / 4, MTA = (DP + 15) / 16, NTB = (DQ + 15) / 16;
  constexpr int NCB = DO * DQ / 16, NRB = DO * DP / 16;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int r = lane & 15, gq = lane >> 4;
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
  // A: T[x_p][(y, y_q)] = sum_{y_p} E_p[x_p][y_p] K[y_p][(y, y_q)], column block cb
  {
    float bc[SP], bn[SP];
    auto ld = [&](int cb, float (&b)[SP]) {
      const int c = 16 * cb + r, y = c / DQ, yq = c - y * DQ;
      const float* col = sV + y * PQS + yq;
#pragma unroll
      for (int s = 0; s < SP; ++s) b[s] = col[(4 * s + gq) * DQ];
    };
    if (wid < NCB) ld(wid, bc);
#pragma unroll
    for (int j = 0; j < (NCB + 3) / 4; ++j) {
      const int cb = wid + 4 * j;
      if (cb < NCB) {
        if (cb + 4 < NCB) ld(cb + 4, bn);
        floatx4 acc[MTA];
#pragma unroll
        for (int mi = 0; mi < MTA; ++mi) acc[mi] = zero;
#pragma unroll
        for (int s = 0; s < SP; ++s)
#pragma unroll
          for (int mi = 0; mi < MTA; ++mi) acc[mi] = __builtin_amdgcn_mfma_f32_16x16x4f32(ea[s][mi], bc[s], acc[mi], 0, 0, 0);
        const int c = 16 * cb + r, y = c / DQ, yq = c - y * DQ;
        float* col = sV + y * PQS + yq;
#pragma unroll
        for (int mi = 0; mi < MTA; ++mi)
          if (16 * mi + 4 * gq + 3 < DP)
#pragma unroll
            for (int i = 0; i < 4; ++i) col[(16 * mi + 4 * gq + i) * DQ] = acc[mi][i];
#pragma unroll
        for (int s = 0; s < SP; ++s) bc[s] = bn[s];
      }
    }
  }
  __syncthreads();
  // B: V[(y, x_p)][x_q] = sum_{y_q} T[(y, x_p)][y_q] E_q[x_q][y_q], row block rb
  {
    float ac[SQ], an[SQ];
    auto ld = [&](int rb, float (&a)[SQ]) {
      const int R = 16 * rb + r, y = R / DP, xp = R - y * DP;
      const float* row = sV + y * PQS + xp * DQ;
#pragma unroll
      for (int s = 0; s < SQ; ++s) a[s] = row[4 * s + gq];
    };
    if (wid < NRB) ld(wid, ac);
#pragma unroll
    for (int j = 0; j < (NRB + 3) / 4; ++j) {
      const int rb = wid + 4 * j;
      if (rb < NRB) {
        if (rb + 4 < NRB) ld(rb + 4, an);
        floatx4 acc[NTB];
#pragma unroll
        for (int ni = 0; ni < NTB; ++ni) acc[ni] = zero;
#pragma unroll
        for (int s = 0; s < SQ; ++s)
#pragma unroll
          for (int ni = 0; ni < NTB; ++ni) acc[ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[s], eb[s][ni], acc[ni], 0, 0, 0);
#pragma unroll
        for (int ni = 0; ni < NTB; ++ni)
          if (16 * ni + r < DQ)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int R2 = 16 * rb + 4 * gq + i, y2 = R2 / DP, xp2 = R2 - y2 * DP;
              sV[y2 * PQS + xp2 * DQ + 16 * ni + r] = acc[ni][i];
            }
#pragma unroll
        for (int s = 0; s < SQ; ++s) ac[s] = an[s];
      }
    }
  }
  __syncthreads();
}

// C0, C1, C2 > 0: the three leg dimensions and the output leg OU known at
// compile time (loop trip counts and strides become constants); all zero:
// read from g.
template <int C0, int C1, int C2, int OU>
__global__ __launch_bounds__(256, 2) void ienv3_kernel(IEnv3Args g) {
  extern __shared__ float smem[];
  constexpr bool CT = C0 > 0;
  const int lo = CT ? OU : g.o, lp = CT ? (OU == 0 ? 1 : 0) : g.p, lq = CT ? (OU == 2 ? 1 : 2) : g.q;
  const int dm0 = CT ? C0 : g.dim[0], dm1 = CT ? C1 : g.dim[1], dm2 = CT ? C2 : g.dim[2];
  const int st0 = CT ? C1 * C2 : g.stride[0], st1 = CT ? C2 : g.stride[1], st2 = CT ? 1 : g.stride[2];
  const int dims[3] = {dm0, dm1, dm2}, strides[3] = {st0, st1, st2};
  const int Do = dims[lo], Dp = dims[lp], Dq = dims[lq];
  const int PQ = Dp * Dq;
  const int PQS = PQ | 1;             // odd row stride: 16 consecutive rows in 16 LDS banks
  float* sV = smem;                   // [Do][PQS]: K_y rows, then V_y rows
  float* sEp = sV + Do * PQS;         // [32][IE_LD] zero-padded E_p[x_p][y_p]
  float* sEq = sEp + 32 * IE_LD;      // [32][IE_LD] zero-padded E_q[x_q][y_q]
  float* sT = sEq + 32 * IE_LD;       // 4 x [32][IE_LD] per-wave tiles
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int r = lane & 15, gq = lane >> 4;
  const int z = blockIdx.x;
  if (z >= g.n) return;  // uniform per workgroup, before any barrier
  int ib = g.pb[z], ik = g.pk[z];
  if (ib < 0 || ib >= g.bra_rows || ik < 0 || ik >= g.ket_rows) {  // clamp and report
    if (tid == 0) atomicOr(g.flag + 2, 1);
    ib = ib < 0 ? 0 : (ib >= g.bra_rows ? g.bra_rows - 1 : ib);
    ik = ik < 0 ? 0 : (ik >= g.ket_rows ? g.ket_rows - 1 : ik);
  }
  const float* __restrict__ bra = g.bra + (int64_t)ib * g.bra_size;
  const float* __restrict__ ket = g.ket + (int64_t)ik * g.ket_size;
  const float* __restrict__ Ep = g.Ep + (int64_t)z * g.ep_stride;
  const float* __restrict__ Eq = g.Eq + (int64_t)z * g.eq_stride;
  float* __restrict__ Eo = g.Eo + (int64_t)z * g.eo_stride;

  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
  float* T = sT + wid * 32 * IE_LD;
  floatx4 acc[2][2] = {{zero, zero}, {zero, zero}};
  const int so = strides[lo], sp = strides[lp], sq = strides[lq];
  int ro[2];
  bool rv[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int xo = 16 * i + r;
    rv[i] = xo < Do;
    ro[i] = rv[i] ? xo * so : 0;
  }
  // compile-time dims of the output leg and the two contracted legs
  constexpr int CDo = OU == 0 ? C0 : (OU == 1 ? C1 : C2);
  constexpr int CDp = OU == 0 ? C1 : C0;
  constexpr int CDq = OU == 2 ? C1 : C2;
  if constexpr (CT) {
    static_assert(C2 % 4 == 0 && (CDp * CDq) % 16 == 0, "compile-time shapes: D_2 % 4 == 0, D_p D_q % 16 == 0");
    // E_o[x_o][y_o] = sum_k Bra[x_o][k] V[y_o][k], k = x_p D_q + x_q, a
    // quarter of the k range per wave.  UK: the last contracted leg is
    // unit-stride in the tensor, so a lane loads its bra rows as 16-byte runs
    // of k (4 consecutive x_q, never crossing an x_p row since D_q % 4 == 0)
    // and MFMA t of a 16-k chunk takes element t of every lane's run, the V
    // operand read the same way (the sum over k is complete whichever k each
    // MFMA sees, as long as A and B agree); otherwise single floats, k = 4 s + gq.
    constexpr bool UK = (OU == 0 || OU == 1) && CDq % 4 == 0 && (CDp * CDq / 4) % 16 == 0;
    constexpr int KW = CDp * CDq / 4;  // k per wave
    const int kbase = KW * wid;
    // ---- every load of the pair in flight at once: the ket, the E_p / E_q
    // fragments, the bra fragments of the last product (raw: padded rows
    // read row 0 through ro); only the ket is waited for before the products
    floatx4 kv[ie_pt<C0 * C1 * C2>];
    ie_load_x<C0 * C1 * C2>(ket, kv);
    float ea[8][2], eb[8][2];
    ie_efrag<CDp>(Ep, ea);
    ie_efrag<CDq>(Eq, eb);
    floatx4 bq[UK ? KW / 16 : 1][2];
    float ac[UK ? 1 : KW / 4][2];
    if constexpr (UK) {
#pragma unroll
      for (int c = 0; c < KW / 16; ++c) {
        const int kk = kbase + 16 * c + 4 * gq;
        const int xp = kk / CDq, xq = kk - xp * CDq;
#pragma unroll
        for (int i = 0; i < 2; ++i) bq[c][i] = *(const floatx4*)(bra + ro[i] + xp * sp + xq);
      }
    } else {
#pragma unroll
      for (int j = 0; j < KW / 4; ++j) {
        const int kk = kbase + 4 * j + gq;
        const int xp = kk / CDq, xq = kk - xp * CDq;
#pragma unroll
        for (int i = 0; i < 2; ++i) ac[j][i] = bra[ro[i] + xp * sp + xq * sq];
      }
    }
    // ---- ket rows K_y in LDS, then V_y = E_p K_y E_q^T
    int ls[3];
    ls[lo] = PQS;
    ls[lp] = CDq;
    ls[lq] = 1;
    ie_store_x<C0, C1, C2>(kv, sV, ls[0], ls[1], ls[2]);
    __syncthreads();
    ie_products_ct<CDo, CDp, CDq>(sV, ea, eb, PQS);
    // ---- the last product, V operands read ahead of the MFMAs; rows x_o,
    // y_o >= D_o of the padded tiles only reach discarded outputs, so their
    // lanes read row D_o - 1 of V instead of being masked
    int yc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) yc[i] = (16 * i + r < CDo ? 16 * i + r : CDo - 1) * PQS;
    if constexpr (UK) {
      float vc[4][2], vn[4][2];
      auto ldv = [&](int c, float (&v)[4][2]) {
        const int kk = kbase + 16 * c + 4 * gq;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < 2; ++i) v[t][i] = sV[yc[i] + kk + t];
      };
      ldv(0, vc);
#pragma unroll
      for (int c = 0; c < KW / 16; ++c) {
        if (c + 1 < KW / 16) ldv(c + 1, vn);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int ni = 0; ni < 2; ++ni)
              acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(bq[c][mi][t], vc[t][ni], acc[mi][ni], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < 2; ++i) vc[t][i] = vn[t][i];
      }
    } else {
      constexpr int SW = KW / 4;  // k-steps per wave
      constexpr int PF = 4;       // V reads this many steps ahead
      float vb[PF + 1][2];        // ring of k-steps j % (PF + 1)
      auto ldv = [&](int j) {
        const int kk = kbase + 4 * j + gq;
#pragma unroll
        for (int i = 0; i < 2; ++i) vb[j % (PF + 1)][i] = sV[yc[i] + kk];
      };
#pragma unroll
      for (int j = 0; j < PF && j < SW; ++j) ldv(j);
#pragma unroll
      for (int j = 0; j < SW; ++j) {
        if (j + PF < SW) ldv(j + PF);
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
          for (int ni = 0; ni < 2; ++ni)
            acc[mi][ni] =
                __builtin_amdgcn_mfma_f32_16x16x4f32(ac[j][mi], vb[j % (PF + 1)][ni], acc[mi][ni], 0, 0, 0);
      }
    }
  } else {
    ie_stage_v(ket, Ep, Eq, sV, sEp, sEq, sT, dm0, dm1, dm2, lo, lp, lq, Do, Dp, Dq, PQS);
    // ---- E_o[x_o][y_o] = sum_k Bra[x_o][k] V[y_o][k], k = x_p * Dq + x_q split over the waves
    const int steps = (PQ + 3) >> 2;
    const int s0 = (steps * wid) >> 2, s1 = (steps * (wid + 1)) >> 2;
    // this lane's k = 4 s + gq as (x_p, x_q), advanced by 4 per step
    int k = 4 * s0 + gq;
    int kp = k / Dq, kq = k - (k / Dq) * Dq;
    // bra fragments eight steps ahead: batch c + 1 is loaded while batch c is multiplied
    constexpr int SB = 8;
    float an[SB][2], ac[SB][2];
    auto load_batch = [&](int sb, float (&dst)[SB][2]) {
#pragma unroll
      for (int j = 0; j < SB; ++j) {
        const bool kv = sb + j < s1 && k < PQ;
        const int ko = kv ? kp * sp + kq * sq : 0;
#pragma unroll
        for (int i = 0; i < 2; ++i) dst[j][i] = bra[ro[i] + ko];  // raw (clamped address); masked at use
        k += 4;
        kq += 4;
        while (kq >= Dq) {
          kq -= Dq;
          ++kp;
        }
      }
    };
    load_batch(s0, ac);
    int kb = 4 * s0 + gq;  // k of the batch being multiplied
    for (int sb = s0; sb < s1; sb += SB) {
      if (sb + SB < s1) load_batch(sb + SB, an);
#pragma unroll
      for (int j = 0; j < SB; ++j) {
        const bool kv = sb + j < s1 && kb < PQ;
        float b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int yo = 16 * i + r;
          b[i] = (kv && yo < Do) ? sV[yo * PQS + kb] : 0.f;
        }
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
          for (int ni = 0; ni < 2; ++ni)
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32((rv[mi] && kv) ? ac[j][mi] : 0.f, b[ni], acc[mi][ni], 0, 0,
                                                               0);
        kb += 4;
      }
#pragma unroll
      for (int j = 0; j < SB; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) ac[j][i] = an[j][i];
    }
  }
  // partial blocks through the per-wave tiles (free now), summed by all threads
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int i = 0; i < 4; ++i) T[(16 * mi + 4 * gq + i) * IE_LD + 16 * ni + r] = acc[mi][ni][i];
  __syncthreads();
  for (int e = tid; e < Do * Do; e += 256) {
    const int xo = e / Do, yo = e - xo * Do;
    const int o = xo * IE_LD + yo;
    Eo[e] = sT[o] + sT[32 * IE_LD + o] + sT[2 * 32 * IE_LD + o] + sT[3 * 32 * IE_LD + o];
  }
}

// Identity-operator effective-Hamiltonian product at the same node type (the
// fitting sweep's per-term local products, Sec. II.C):
//   Y[z][x_0, x_1, x_2] = sum E_0[x_0][y_0] E_1[x_1][y_1] E_2[x_2][y_2] X[xr][y_0, y_1, y_2],
// xr = x_ids[z] (or z), environment slot z.  One workgroup per item: the shared
// phase with leg 0 as the row leg (V_y = E_1 K_y E_2^T), then
// Y = E_0 V (M = D_0, N = D_1 D_2, K = D_0), the N columns split over the waves
// and written straight to Y (rows of D_1 D_2 contiguous floats).
template <int C0, int C1, int C2>
__global__ __launch_bounds__(256, 2) void iheff3_kernel(IHeff3Args g) {
  extern __shared__ float smem[];
  constexpr int DU = C0;  // > 0: dims known at compile time
  const int dm0 = DU ? C0 : g.dim[0], dm1 = DU ? C1 : g.dim[1], dm2 = DU ? C2 : g.dim[2];
  const int Do = dm0, Dp = dm1, Dq = dm2;
  const int PQ = Dp * Dq;
  const int PQS = PQ | 1;
  float* sV = smem;
  float* sEp = sV + Do * PQS;
  float* sEq = sEp + 32 * IE_LD;
  float* sT = sEq + 32 * IE_LD;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int r = lane & 15, gq = lane >> 4;
  const int z = blockIdx.x;
  if (z >= g.n) return;  // uniform per workgroup, before any barrier
  int xr = g.x_ids ? g.x_ids[z] : z;
  if (xr < 0 || xr >= g.x_rows) {  // clamp and report
    if (tid == 0) atomicOr(g.flag + 2, 1);
    xr = xr < 0 ? 0 : g.x_rows - 1;
  }
  const float* __restrict__ X = g.X + (int64_t)xr * g.x_size;
  const float* __restrict__ E0 = g.E[0] + (int64_t)z * g.e_stride[0];
  float* __restrict__ Y = g.Y + (int64_t)z * g.y_stride;
  const float* __restrict__ E1 = g.E[1] + (int64_t)z * g.e_stride[1];
  const float* __restrict__ E2 = g.E[2] + (int64_t)z * g.e_stride[2];
  float e0[8][2];  // E_0 fragments e0[s][i] = E_0[16 i + r][4 s + gq], zero outside
  if constexpr (DU > 0) {
    static_assert(C2 % 4 == 0, "compile-time shapes: D_2 % 4 == 0");
    // every load of the item in flight at once, the tensor waited for first
    floatx4 kv[ie_pt<C0 * C1 * C2>];
    ie_load_x<C0 * C1 * C2>(X, kv);
    float ea[8][2], eb[8][2];
    ie_efrag<C1>(E1, ea);
    ie_efrag<C2>(E2, eb);
    ie_efrag<C0>(E0, e0);
    ie_store_x<C0, C1, C2>(kv, sV, PQS, C2, 1);
    __syncthreads();
    ie_products_ct<C0, C1, C2>(sV, ea, eb, PQS);
    // Y = E_0 V: column tiles of 16 dealt to the waves, the next tile's V
    // operands read before the current tile's MFMAs
    constexpr int NT = C1 * C2 / 16, S0 = C0 / 4, MT = (C0 + 15) / 16;
    static_assert((C1 * C2) % 16 == 0 && C0 % 4 == 0, "compile-time output tiles");
    const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
    float bc[S0], bn[S0];
    auto ld = [&](int nt, float (&b)[S0]) {
#pragma unroll
      for (int s = 0; s < S0; ++s) b[s] = sV[(4 * s + gq) * PQS + 16 * nt + r];
    };
    if (wid < NT) ld(wid, bc);
#pragma unroll
    for (int j = 0; j < (NT + 3) / 4; ++j) {
      const int nt = wid + 4 * j;
      if (nt < NT) {
        if (nt + 4 < NT) ld(nt + 4, bn);
        floatx4 acc[MT];
#pragma unroll
        for (int mi = 0; mi < MT; ++mi) acc[mi] = zero;
#pragma unroll
        for (int s = 0; s < S0; ++s)
#pragma unroll
          for (int mi = 0; mi < MT; ++mi) acc[mi] = __builtin_amdgcn_mfma_f32_16x16x4f32(e0[s][mi], bc[s], acc[mi], 0, 0, 0);
        const int n = 16 * nt + r;
#pragma unroll
        for (int mi = 0; mi < MT; ++mi)
          if (16 * mi + 4 * gq + 3 < C0)
#pragma unroll
            for (int i = 0; i < 4; ++i) Y[(16 * mi + 4 * gq + i) * PQ + n] = acc[mi][i];
#pragma unroll
        for (int s = 0; s < S0; ++s) bc[s] = bn[s];
      }
    }
    return;
  } else {
    ie_stage_v(X, E1, E2, sV, sEp, sEq, sT, dm0, dm1, dm2, 0, 1, 2, Do, Dp, Dq, PQS);
    // E_0 zero-padded into the (now free) tile area
    float* sE0 = sT;
    for (int e = tid; e < 32 * 32; e += 256) {
      const int a = e >> 5, b = e & 31;
      sE0[a * IE_LD + b] = (a < Do && b < Do) ? E0[a * Do + b] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i) e0[s][i] = sE0[(16 * i + r) * IE_LD + 4 * s + gq];
  }
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
  const int ntiles = (PQ + 15) >> 4, ksteps = (Do + 3) >> 2;
  for (int nt = wid; nt < ntiles; nt += 4) {
    const int n = 16 * nt + r;
    floatx4 acc[2] = {zero, zero};
#pragma unroll
    for (int s = 0; s < (DU ? (C0 + 3) / 4 : 8); ++s) {
      if (!DU && s >= ksteps) break;
      const int k = 4 * s + gq;
      const float b = (k < Do && n < PQ) ? sV[k * PQS + n] : 0.f;
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
        acc[mi] = __builtin_amdgcn_mfma_f32_16x16x4f32(e0[s][mi], b, acc[mi], 0, 0, 0);
    }
    if (n < PQ) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int x0 = 16 * mi + 4 * gq + i;
          if (x0 < Do) Y[x0 * PQ + n] = acc[mi][i];
        }
    }
  }
}

hipError_t launch_iheff3(const IHeff3Args& a, hipStream_t s) {
  const size_t bytes = ienv3_lds_bytes(a.dim[0], a.dim[1], a.dim[2]);
  auto set_lds = [](const void* f) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)IENV3_LDS_MAX) == hipSuccess;
  };
  static const bool attr = set_lds(reinterpret_cast<const void*>(&iheff3_kernel<24, 24, 24>)) &&
                           set_lds(reinterpret_cast<const void*>(&iheff3_kernel<24, 8, 8>)) &&
                           set_lds(reinterpret_cast<const void*>(&iheff3_kernel<0, 0, 0>));
  if (!attr || bytes > IENV3_LDS_MAX) return hipErrorInvalidValue;
  const dim3 grid((unsigned)a.n), blk(256);
  // the compile-time shapes load the tensor as 16-byte runs
  const bool al = (uintptr_t)a.X % 16 == 0 && a.x_size % 4 == 0;
  if (al && a.dim[0] == 24 && a.dim[1] == 24 && a.dim[2] == 24)
    hipLaunchKernelGGL((iheff3_kernel<24, 24, 24>), grid, blk, bytes, s, a);
  else if (al && a.dim[0] == 24 && a.dim[1] == 8 && a.dim[2] == 8)
    hipLaunchKernelGGL((iheff3_kernel<24, 8, 8>), grid, blk, bytes, s, a);
  else
    hipLaunchKernelGGL((iheff3_kernel<0, 0, 0>), grid, blk, bytes, s, a);
  return hipGetLastError();
}

size_t ienv3_lds_bytes(int Do, int Dp, int Dq) {
  return sizeof(float) * ((size_t)Do * ((Dp * Dq) | 1) + 6 * 32 * IE_LD);
}

hipError_t launch_ienv3(const IEnv3Args& a, hipStream_t s) {
  const size_t bytes = ienv3_lds_bytes(a.dim[a.o], a.dim[a.p], a.dim[a.q]);
  auto set_lds = [](const void* f) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)IENV3_LDS_MAX) == hipSuccess;
  };
  static const bool attr = set_lds(reinterpret_cast<const void*>(&ienv3_kernel<24, 24, 24, 0>)) &&
                           set_lds(reinterpret_cast<const void*>(&ienv3_kernel<24, 24, 24, 1>)) &&
                           set_lds(reinterpret_cast<const void*>(&ienv3_kernel<24, 24, 24, 2>)) &&
                           set_lds(reinterpret_cast<const void*>(&ienv3_kernel<24, 8, 8, 0>)) &&
                           set_lds(reinterpret_cast<const void*>(&ienv3_kernel<24, 8, 8, 1>)) &&
                           set_lds(reinterpret_cast<const void*>(&ienv3_kernel<24, 8, 8, 2>)) &&
                           set_lds(reinterpret_cast<const void*>(&ienv3_kernel<0, 0, 0, 0>));
  if (!attr || bytes > IENV3_LDS_MAX) return hipErrorInvalidValue;
  const dim3 grid((unsigned)a.n), blk(256);
  // the compile-time shapes load the tensors as 16-byte runs
  const bool al = ((uintptr_t)a.bra | (uintptr_t)a.ket) % 16 == 0 && a.bra_size % 4 == 0 && a.ket_size % 4 == 0;
#define IENV3_CASE(A0, A1, A2)                                                                      \
  if (al && a.dim[0] == A0 && a.dim[1] == A1 && a.dim[2] == A2) {                                   \
    if (a.o == 0) hipLaunchKernelGGL((ienv3_kernel<A0, A1, A2, 0>), grid, blk, bytes, s, a);        \
    else if (a.o == 1) hipLaunchKernelGGL((ienv3_kernel<A0, A1, A2, 1>), grid, blk, bytes, s, a);   \
    else hipLaunchKernelGGL((ienv3_kernel<A0, A1, A2, 2>), grid, blk, bytes, s, a);                 \
    return hipGetLastError();                                                                       \
  }
  // the binary-tree nodes: uniform 24 bonds, and 24 to the parent with two 8-bond leaves
  IENV3_CASE(24, 24, 24)
  IENV3_CASE(24, 8, 8)
#undef IENV3_CASE
  hipLaunchKernelGGL((ienv3_kernel<0, 0, 0, 0>), grid, blk, bytes, s, a);
  return hipGetLastError();
}

}  // namespace ttn
