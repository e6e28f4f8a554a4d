// C ABI: Rayleigh-Ritz, QR gauge moves, node norms and scaling.
#include <hip/hip_runtime.h>

#include <cstring>
#include <sstream>

#include <string>

#include "internal.h"

using namespace ttn;

namespace ttn {
hipError_t launch_rr(int batch, const int32_t* d_m, int ld, const double* H, const double* S, int nev, double drop_tol,
                     int allow_svqb, double* evals, double* V, int32_t* rank, double* scratch, int* flag,
                     hipStream_t s);
hipError_t launch_qr(int ctype, void* X, int64_t size, const int32_t* roff, int m, int n, int64_t cstride, double* work,
                     double* R, int nz, int* flag, hipStream_t s);
const char* qr_path_name(int m, int n);
bool absorb_in_place(int m, int n);
hipError_t launch_absorb(int ctype, const void* X, int64_t size, const int32_t* roff, int m, int n, int64_t cstride,
                         const double* R, void* Y, int nz, hipStream_t s);
hipError_t launch_norms2(int ctype, const void* X, int64_t n, int nz, double* out, hipStream_t s);
hipError_t launch_scale(int ctype, void* X, int64_t n, int nz, const double* sc, hipStream_t s);
hipError_t launch_scatter2(int n, const int32_t* ia, const int32_t* ib, const double* vals, double* out, hipStream_t s);
hipError_t launch_vscale(int n, const double* x, double a, double* y, hipStream_t s);
hipError_t launch_vsqrt(const double* x, double* y, int n, hipStream_t s);
hipError_t launch_vgather(const int32_t* idx, const double* src, int src_n, double fill, double* dst, int n, int* flag,
                          hipStream_t s);
hipError_t launch_convert(int sdt, const void* x, int ddt, void* y, int64_t n, hipStream_t s);
hipError_t launch_normalize(int ctype, void* X, int64_t n, int nz, double* norms, hipStream_t s);

ttn_status api_fail(ttn_ctx* ctx, ttn_status code, const std::string& msg);

// offsets of the "rest" rows of node u's tensor when leg `leg` is the column
// index (cached per shape on the context); returns a device table
const int32_t* leg_rows_table(ttn_ctx* ctx, const std::vector<int>& dims, int leg, int64_t& cstride, int& m,
                              ttn_status& code) {
  std::ostringstream k;
  k << "rows";
  for (int d : dims) k << ":" << d;
  k << "@" << leg;
  const int nd = (int)dims.size();
  std::vector<int64_t> st(nd, 1);
  for (int i = nd - 2; i >= 0; --i) st[i] = st[i + 1] * dims[i + 1];
  cstride = st[leg];
  int64_t rows = 1;
  for (int i = 0; i < nd; ++i)
    if (i != leg) rows *= dims[i];
  m = (int)rows;
  auto it = ctx->tables.find(k.str());
  if (it != ctx->tables.end()) return it->second;
  std::vector<int32_t> off((size_t)rows, 0);
  std::vector<int> idx(nd, 0);
  for (int64_t r = 0; r < rows; ++r) {
    int64_t o = 0;
    for (int i = 0; i < nd; ++i) o += (int64_t)idx[i] * st[i];
    off[(size_t)r] = (int32_t)o;
    for (int i = nd - 1; i >= 0; --i) {
      if (i == leg) continue;
      if (++idx[i] < dims[i]) break;
      idx[i] = 0;
    }
  }
  const int32_t* d = pool_upload(ctx, std::move(off), code);
  if (!d) return nullptr;
  ctx->tables[k.str()] = d;
  return d;
}
}  // namespace ttn

extern "C" {

ttn_status rayleigh_ritz(ttn_ctx* ctx, int32_t batch, const int32_t* m, int32_t ld, const double* H, const double* S,
                         int32_t nev, double drop_tol, int32_t allow_svqb, double* evals, double* V,
                         int32_t* rank_out) {
  if (!ctx || !m || !H || !S || !evals || !V || !rank_out) return api_fail(ctx, TTN_E_ARG, "null argument");
  if (batch < 0 || ld < 1 || ld > 512 || nev < 1 || nev > ld) return api_fail(ctx, TTN_E_ARG, "bad sizes (ld <= 512)");
  if (!(drop_tol >= 0)) return api_fail(ctx, TTN_E_ARG, "drop_tol must be >= 0");
  for (int b = 0; b < batch; ++b)
    if (m[b] < 1 || m[b] > ld) return api_fail(ctx, TTN_E_ARG, "m[b] outside [1, ld]");
  if (batch == 0) return TTN_OK;
  const size_t need = (size_t)batch * 4 * ld * ld * sizeof(double) + 256 + (size_t)batch * sizeof(int32_t);
  if (need > ctx->ws_bytes) return api_fail(ctx, TTN_E_WORKSPACE, "workspace too small for Rayleigh-Ritz");
  ctx->ws_last_plan = nullptr;
  int32_t* d_m = (int32_t*)ctx->ws;
  double* scratch = (double*)((char*)ctx->ws + 256 + (((size_t)batch * sizeof(int32_t) + 255) / 256) * 256);
  if (hipMemcpyAsync(d_m, m, (size_t)batch * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
    return api_fail(ctx, TTN_E_DEVICE, "copy of m failed");
  ttn_prof_rec* pr = prof_begin(ctx, "rr", "rr_kernel", 0.0, 2.0 * 8.0 * batch * (double)ld * ld, batch);
  hipError_t e = launch_rr(batch, d_m, ld, H, S, nev, drop_tol, allow_svqb, evals, V, rank_out, scratch, ctx->d_flag,
                           ctx->stream);
  prof_end(ctx, pr);
  if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
  return TTN_OK;
}

ttn_status ttn_block_move_centre(ttn_ctx* ctx, ttn_block* b, int32_t u, int32_t v) {
  if (!ctx || !b) return api_fail(ctx, TTN_E_ARG, "null argument");
  const ttn_tree* t = b->t;
  if (u < 0 || u >= t->n || t->leg_of(u, v) < 0) return api_fail(ctx, TTN_E_ARG, "v is not a neighbour of u");
  const int ct = b->dt == TTN_F64 ? 0 : 1;
  const size_t es = ct == 0 ? 8 : 4;
  const std::vector<int> du = b->legdims(u), dv = b->legdims(v);
  const int lu = t->leg_of(u, v), lv = t->leg_of(v, u);
  int64_t cs_u = 0, cs_v = 0;
  int m_u = 0, m_v = 0;
  ttn_status code = TTN_OK;
  const int32_t* ru = leg_rows_table(ctx, du, lu, cs_u, m_u, code);
  if (!ru) return code;
  const int32_t* rv = leg_rows_table(ctx, dv, lv, cs_v, m_v, code);
  if (!rv) return code;
  const int n = du[lu];
  if (n > 512) return api_fail(ctx, TTN_E_SHAPE, "bond dimension above 512");
  if (m_u < n) return api_fail(ctx, TTN_E_SHAPE, "QR needs rows >= bond (bond exceeds the tensor's other legs)");
  const int k = b->k;
  const size_t work = (size_t)k * 2 * m_u * n * sizeof(double);
  const size_t rbytes = (size_t)k * (n * n + n) * sizeof(double);  // R blocks, then tau per reflector
  const size_t ybytes = (size_t)k * b->size[v] * es;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  if (al(work) + al(rbytes) + al(ybytes) > ctx->ws_bytes) return api_fail(ctx, TTN_E_WORKSPACE, "workspace too small for QR");
  ctx->ws_last_plan = nullptr;
  double* wk = (double*)ctx->ws;
  double* R = (double*)((char*)ctx->ws + al(work));
  void* Y = (char*)ctx->ws + al(work) + al(rbytes);
  // Householder QR with explicit Q: 4 m n^2 - 4 n^3 / 3 flops per state; the
  // tensor is read and written once, R written once
  const double fq = 4.0 * m_u * (double)n * n - 4.0 * (double)n * n * n / 3.0;
  const std::string qkey = "qr:" + std::to_string(m_u) + "x" + std::to_string(n);
  ttn_prof_rec* pr = prof_begin(ctx, qkey.c_str(), qr_path_name(m_u, n), fq * k, (double)k * (2.0 * m_u * n * es + 8.0 * n * n), k);
  hipError_t e = launch_qr(ct, b->ptr[u], b->size[u], ru, m_u, n, cs_u, wk, R, k, ctx->d_flag, ctx->stream);
  prof_end(ctx, pr);
  if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
  const std::string akey = "absorb:" + std::to_string(m_v) + "x" + std::to_string(n);
  pr = prof_begin(ctx, akey.c_str(), "absorb_kernel", 2.0 * m_v * (double)n * n * k,
                  (double)k * (2.0 * m_v * n * es + 8.0 * n * n), k);
  const bool in_place = absorb_in_place(m_v, n);
  e = launch_absorb(ct, b->ptr[v], b->size[v], rv, m_v, n, cs_v, R, in_place ? b->ptr[v] : Y, k, ctx->stream);
  prof_end(ctx, pr);
  if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
  if (!in_place &&
      hipMemcpyAsync(b->ptr[v], Y, (size_t)k * b->size[v] * es, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess)
    return api_fail(ctx, TTN_E_DEVICE, "copy back failed");
  return TTN_OK;
}

ttn_status ttn_block_scale_node(ttn_ctx* ctx, ttn_block* b, int32_t u, const double* scale) {
  if (!ctx || !b || !scale || u < 0 || u >= b->t->n) return api_fail(ctx, TTN_E_ARG, "bad arguments");
  hipError_t e = launch_scale(b->dt == TTN_F64 ? 0 : 1, b->ptr[u], b->size[u], b->k, scale, ctx->stream);
  if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
  return TTN_OK;
}

ttn_status ttn_block_node_norms2(ttn_ctx* ctx, const ttn_block* b, int32_t u, double* out) {
  if (!ctx || !b || !out || u < 0 || u >= b->t->n) return api_fail(ctx, TTN_E_ARG, "bad arguments");
  hipError_t e = launch_norms2(b->dt == TTN_F64 ? 0 : 1, b->ptr[u], b->size[u], b->k, out, ctx->stream);
  if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
  return TTN_OK;
}

ttn_status ttn_block_normalize_node(ttn_ctx* ctx, ttn_block* b, int32_t u, double* norms_out) {
  if (!ctx || !b || u < 0 || u >= b->t->n) return api_fail(ctx, TTN_E_ARG, "bad arguments");
  hipError_t e = launch_normalize(b->dt == TTN_F64 ? 0 : 1, b->ptr[u], b->size[u], b->k, norms_out, ctx->stream);
  if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
  return TTN_OK;
}

ttn_status ttn_scatter_sym(ttn_ctx* ctx, int32_t n, const int32_t* idx_a, const int32_t* idx_b, const double* vals,
                           double* out) {
  if (!ctx || n < 0 || (n > 0 && (!idx_a || !idx_b || !vals || !out))) return api_fail(ctx, TTN_E_ARG, "bad arguments");
  hipError_t e = launch_scatter2(n, idx_a, idx_b, vals, out, ctx->stream);
  if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
  return TTN_OK;
}

ttn_status ttn_vec_sqrt(ttn_ctx* ctx, int32_t n, const double* x, double* y) {
  if (!ctx || n < 0 || (n > 0 && (!x || !y))) return api_fail(ctx, TTN_E_ARG, "bad arguments");
  hipError_t e = launch_vsqrt(x, y, n, ctx->stream);
  if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
  return TTN_OK;
}

ttn_status ttn_vec_gather(ttn_ctx* ctx, int32_t n, const int32_t* idx, const double* src, int32_t src_n, double fill,
                          double* dst) {
  if (!ctx || n < 0 || src_n < 0 || (n > 0 && (!idx || !dst || (src_n > 0 && !src))))
    return api_fail(ctx, TTN_E_ARG, "bad arguments");
  hipError_t e = launch_vgather(idx, src, src_n, fill, dst, n, ctx->d_flag, ctx->stream);
  if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
  return TTN_OK;
}

ttn_status ttn_block_convert(ttn_ctx* ctx, const ttn_block* src, ttn_block* dst, int32_t rows) {
  if (!ctx || !src || !dst) return api_fail(ctx, TTN_E_ARG, "null argument");
  if (src->t->parent != dst->t->parent || src->t->phys != dst->t->phys || src->D != dst->D)
    return api_fail(ctx, TTN_E_SHAPE, "blocks differ in tree or bonds");
  if (rows < 0 || rows > src->k || rows > dst->k) return api_fail(ctx, TTN_E_ARG, "rows outside both blocks");
  if ((src->dt != TTN_F64 && src->dt != TTN_F32) || (dst->dt != TTN_F64 && dst->dt != TTN_F32))
    return api_fail(ctx, TTN_E_DTYPE, "blocks must be FP64 or FP32");
  const int sdt = src->dt == TTN_F64 ? 0 : 1, ddt = dst->dt == TTN_F64 ? 0 : 1;
  for (int u = 0; u < src->t->n; ++u) {
    hipError_t e = launch_convert(sdt, src->ptr[u], ddt, dst->ptr[u], (int64_t)rows * src->size[u], ctx->stream);
    if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
  }
  return TTN_OK;
}

ttn_status ttn_vec_scale(ttn_ctx* ctx, int32_t n, const double* x, double alpha, double* y) {
  if (!ctx || n < 0 || (n > 0 && (!x || !y))) return api_fail(ctx, TTN_E_ARG, "bad arguments");
  hipError_t e = launch_vscale(n, x, alpha, y, ctx->stream);
  if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
  return TTN_OK;
}

}  // extern "C"
