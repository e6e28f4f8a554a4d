// C ABI of the learned local preconditioner: a 3-layer MLP 128 -> 256 -> 256
// -> 64 with SiLU activations (forward, backward, MSE loss, Adam), its tile
// features, and the dense GEMMs it needs (on the offset-table matrix-core
// engine; BF16 compute rounds FP32 master weights to bfloat16 when staging,
// accumulation is FP32).
#include <hip/hip_runtime.h>

#include <sstream>

#include "internal.h"

using namespace ttn;

namespace ttn {
hipError_t launch_bias_act(float* pre, float* post, const float* bias, int n, int w, int act, hipStream_t s);
hipError_t launch_dact(float* g, const float* pre, int64_t total, hipStream_t s);
hipError_t launch_colsum(const float* g, int n, int w, float* db, hipStream_t s);
hipError_t launch_mse(const float* Y, const float* Tg, float* dY, int64_t total, double* loss, hipStream_t s);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);
hipError_t launch_zero_double(double* x, hipStream_t s);
hipError_t launch_features(int ctype, const void* b, const void* d, int64_t n, int nz, double* scales, float* X,
                           hipStream_t s);
hipError_t launch_targets(int ctype, const void* y, const void* b, const void* d, int64_t n, int nz,
                          const double* scales, float* Yt, hipStream_t s);

// C[M][N] (+)= op(A) op(B), row-major; ta: A stored [K][M]; tb: B stored [N][K]
ttn_status dense_gemm(ttn_ctx* ctx, int ct, int M, int N, int K, const float* A, bool ta, const float* B, bool tb,
                      float* C, bool accum) {
  std::ostringstream key;
  key << "dense:" << M << ":" << N << ":" << K << ":" << ta << tb;
  const int32_t* tab = nullptr;
  auto it = ctx->tables.find(key.str());
  if (it != ctx->tables.end()) {
    tab = it->second;
  } else {
    std::vector<int32_t> h;
    auto push = [&](int n, int64_t stride) {
      for (int i = 0; i < n; ++i) h.push_back((int32_t)(i * stride));
      while (h.size() % 16) h.push_back(0);
    };
    push(M, ta ? 1 : K);   // a_om
    push(K, ta ? M : 1);   // a_ok
    push(K, tb ? 1 : N);   // b_ok
    push(N, tb ? K : 1);   // b_on
    push(M, N);            // c_om
    push(N, 1);            // c_on
    if ((int64_t)M * K >= INT32_MAX || (int64_t)K * N >= INT32_MAX || (int64_t)M * N >= INT32_MAX)
      return api_fail(ctx, TTN_E_SHAPE, "dense GEMM too large for 32-bit offsets");
    ttn_status code = TTN_OK;
    tab = pool_upload(ctx, std::move(h), code);
    if (!tab) return code;
    ctx->tables[key.str()] = tab;
  }
  auto pad = [](int n) { return (n + 15) / 16 * 16; };
  GemmDesc g;
  g.M = M;
  g.N = N;
  g.K = K;
  int off = 0;
  g.a_om = tab + off;
  off += pad(M);
  g.a_ok = tab + off;
  off += pad(K);
  g.b_ok = tab + off;
  off += pad(K);
  g.b_on = tab + off;
  off += pad(N);
  g.c_om = tab + off;
  off += pad(M);
  g.c_on = tab + off;
  g.a_mfast = ta;
  g.b_nfast = !tb;
  g.tile = (M >= 128 && N >= 128) ? 0 : ((M >= 128) ? 2 : (N >= 128 ? 3 : 1));
  OpAddr a, b, c;
  a.base = A;
  a.shared = true;
  b.base = B;
  b.shared = true;
  c.base = C;
  c.shared = true;
  Epilogue ep;
  ep.accum = accum;
  ctx->flops_done += 2.0 * M * N * K;
  hipError_t e = launch_gemm(ct, g, a, b, c, ep, 0, 1, ctx->d_flag, ctx->stream);
  if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
  return TTN_OK;
}
}  // namespace ttn

namespace {
constexpr int IN = 128, HID = 256, OUT = 64;
constexpr int64_t OW1 = 0, OB1 = OW1 + IN * HID, OW2 = OB1 + HID, OB2 = OW2 + HID * HID, OW3 = OB2 + HID,
                  OB3 = OW3 + HID * OUT, NPAR = OB3 + OUT;

int mlp_ct(ttn_dtype compute) { return compute == TTN_BF16 ? 2 : 1; }

#define HIPL(ctx, e)                                                                   \
  do {                                                                                 \
    hipError_t _e = (e);                                                               \
    if (_e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(_e));   \
  } while (0)
}  // namespace

extern "C" {

int64_t ttn_mlp_num_params(void) { return NPAR; }

ttn_status ttn_mlp_forward(ttn_ctx* ctx, const float* params, int32_t n, const float* X, float* Y, float* acts,
                           ttn_dtype compute) {
  if (!ctx || !params || !X || !Y || n < 0) return api_fail(ctx, TTN_E_ARG, "bad MLP arguments");
  if (compute == TTN_F64) return api_fail(ctx, TTN_E_DTYPE, "MLP computes in FP32 or BF16");
  if (n == 0) return TTN_OK;
  const int ct = mlp_ct(compute);
  // activations: pre1, post1, pre2, post2 (each n x 256); workspace when not kept
  float* A = acts;
  if (!A) {
    if ((size_t)n * 4 * HID * 4 > ctx->ws_bytes) return api_fail(ctx, TTN_E_WORKSPACE, "workspace too small for MLP");
    ctx->ws_last_plan = nullptr;
    A = (float*)ctx->ws;
  }
  float *pre1 = A, *post1 = A + (int64_t)n * HID, *pre2 = A + 2 * (int64_t)n * HID, *post2 = A + 3 * (int64_t)n * HID;
  ttn_status r = dense_gemm(ctx, ct, n, HID, IN, X, false, params + OW1, false, pre1, false);
  if (r) return r;
  HIPL(ctx, launch_bias_act(pre1, post1, params + OB1, n, HID, 1, ctx->stream));
  r = dense_gemm(ctx, ct, n, HID, HID, post1, false, params + OW2, false, pre2, false);
  if (r) return r;
  HIPL(ctx, launch_bias_act(pre2, post2, params + OB2, n, HID, 1, ctx->stream));
  r = dense_gemm(ctx, ct, n, OUT, HID, post2, false, params + OW3, false, Y, false);
  if (r) return r;
  HIPL(ctx, launch_bias_act(Y, Y, params + OB3, n, OUT, 0, ctx->stream));
  return TTN_OK;
}

ttn_status ttn_mlp_backward(ttn_ctx* ctx, const float* params, int32_t n, const float* X, const float* acts,
                            const float* dY, float* grads, ttn_dtype compute) {
  if (!ctx || !params || !X || !acts || !dY || !grads || n < 1) return api_fail(ctx, TTN_E_ARG, "bad MLP arguments");
  if (compute == TTN_F64) return api_fail(ctx, TTN_E_DTYPE, "MLP computes in FP32 or BF16");
  const int ct = mlp_ct(compute);
  if ((size_t)n * 2 * HID * 4 > ctx->ws_bytes) return api_fail(ctx, TTN_E_WORKSPACE, "workspace too small for MLP");
  const float *pre1 = acts, *post1 = acts + (int64_t)n * HID, *pre2 = acts + 2 * (int64_t)n * HID,
              *post2 = acts + 3 * (int64_t)n * HID;
  ctx->ws_last_plan = nullptr;
  float* d2 = (float*)ctx->ws;
  float* d1 = d2 + (int64_t)n * HID;
  // layer 3
  ttn_status r = dense_gemm(ctx, ct, HID, OUT, n, post2, true, dY, false, grads + OW3, false);
  if (r) return r;
  HIPL(ctx, launch_colsum(dY, n, OUT, grads + OB3, ctx->stream));
  r = dense_gemm(ctx, ct, n, HID, OUT, dY, false, params + OW3, true, d2, false);
  if (r) return r;
  HIPL(ctx, launch_dact(d2, pre2, (int64_t)n * HID, ctx->stream));
  // layer 2
  r = dense_gemm(ctx, ct, HID, HID, n, post1, true, d2, false, grads + OW2, false);
  if (r) return r;
  HIPL(ctx, launch_colsum(d2, n, HID, grads + OB2, ctx->stream));
  r = dense_gemm(ctx, ct, n, HID, HID, d2, false, params + OW2, true, d1, false);
  if (r) return r;
  HIPL(ctx, launch_dact(d1, pre1, (int64_t)n * HID, ctx->stream));
  // layer 1
  r = dense_gemm(ctx, ct, IN, HID, n, X, true, d1, false, grads + OW1, false);
  if (r) return r;
  HIPL(ctx, launch_colsum(d1, n, HID, grads + OB1, ctx->stream));
  return TTN_OK;
}

ttn_status ttn_mlp_loss(ttn_ctx* ctx, int32_t n, const float* Y, const float* T, float* dY, double* loss) {
  if (!ctx || !Y || !T || !dY || !loss || n < 1) return api_fail(ctx, TTN_E_ARG, "bad loss arguments");
  HIPL(ctx, launch_zero_double(loss, ctx->stream));
  HIPL(ctx, launch_mse(Y, T, dY, (int64_t)n * OUT, loss, ctx->stream));
  return TTN_OK;
}

ttn_status ttn_mlp_adam(ttn_ctx* ctx, float* params, float* m, float* v, const float* grads, float lr, float beta1,
                        float beta2, float eps, int32_t step) {
  if (!ctx || !params || !m || !v || !grads || step < 1) return api_fail(ctx, TTN_E_ARG, "bad Adam arguments");
  HIPL(ctx, launch_adam(params, m, v, grads, NPAR, lr, beta1, beta2, eps, step, ctx->stream));
  return TTN_OK;
}

ttn_status ttn_precond_features(ttn_ctx* ctx, int32_t k, int64_t n, ttn_dtype storage, const void* b, const void* d,
                                double* scales, float* X) {
  if (!ctx || !b || !d || !scales || !X || k < 0 || n < 1) return api_fail(ctx, TTN_E_ARG, "bad feature arguments");
  if (k == 0) return TTN_OK;
  HIPL(ctx, launch_features(storage == TTN_F64 ? 0 : 1, b, d, n, k, scales, X, ctx->stream));
  return TTN_OK;
}

ttn_status ttn_precond_targets(ttn_ctx* ctx, int32_t k, int64_t n, ttn_dtype storage, const void* y, const void* b,
                               const void* d, const double* scales, float* T) {
  if (!ctx || !y || !b || !d || !scales || !T || k < 0 || n < 1)
    return api_fail(ctx, TTN_E_ARG, "bad target arguments");
  if (k == 0) return TTN_OK;
  HIPL(ctx, launch_targets(storage == TTN_F64 ? 0 : 1, y, b, d, n, k, scales, T, ctx->stream));
  return TTN_OK;
}

}  // extern "C"
