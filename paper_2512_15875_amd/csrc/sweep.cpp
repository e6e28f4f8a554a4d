// C ABI: sweeps of local solves over the tree (ALS for (H - s) y = phi,
// Sec. II.C.3, and variational fitting of sums sum_i c_i O_i phi_i,
// Sec. II.C.2), one local step per sweep_step call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <sstream>

#include "internal.h"

using namespace ttn;

namespace ttn {
ttn_status api_fail(ttn_ctx* ctx, ttn_status code, const std::string& msg);
ttn_status heff_apply_rows(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_envs* envs, int32_t node,
                           int32_t k, const int32_t* pair_ids, const int32_t* x_ids, const int32_t* y_ids,
                           int32_t y_rows, const double* shift, const double* alpha, const void* X, int32_t x_rows,
                           void* Y, uint32_t flags, ttn_dtype compute);
hipError_t launch_minres_init(int ctype, const void* b, const void* Ax, void* v, void* vprev, void* d1, void* d2,
                              int64_t n, int k, double rtol, MinresState* st, int32_t* active, hipStream_t s);
hipError_t launch_minres_count(const MinresState* st, int k, int32_t* active, hipStream_t s);
hipError_t launch_minres_step(int ctype, void* x, void* v, void* vprev, void* p, const void* dp, void* dpp, int64_t n,
                              int k, MinresState* st, hipStream_t s);
hipError_t launch_precond_scale(int ctype, const void* d, void* dsq, int64_t n, int k, int mode, double damp,
                                hipStream_t s);
hipError_t launch_ew_mul(int ctype, const void* a, const void* b, void* out, int64_t n, const int32_t* gate,
                         hipStream_t s);
hipError_t launch_ew_div(int ctype, const void* a, const void* b, void* out, int64_t n, hipStream_t s);
hipError_t launch_minres_report(const MinresState* st, int k, int32_t* iters, double* resid, int32_t* n_active,
                                hipStream_t s);
hipError_t launch_diag_solve(int ctype, const void* b, const void* dg, void* y, int64_t n, hipStream_t s);
hipError_t launch_gather_coef(const double* coef, const int32_t* perm, int n, double* out, hipStream_t s);
hipError_t launch_seg_sum(int ctype, const void* S, const int32_t* ptr, const int32_t* terms, const double* coef,
                          void* y, int64_t n, int k, bool accumulate_first, hipStream_t s);
hipError_t launch_axpy_rows(int ctype, const void* x, void* y, int64_t n, hipStream_t s);
hipError_t launch_resid_zero(int ctype, const void* b, const void* p, void* r, void* zero, int64_t n, hipStream_t s);
hipError_t launch_features(int ctype, const void* b, const void* d, int64_t n, int nz, double* scales, float* X,
                           hipStream_t s);
hipError_t launch_targets(int ctype, const void* y, const void* b, const void* d, int64_t n, int nz,
                          const double* scales, float* Yt, hipStream_t s);
hipError_t launch_untile(int ctype, const float* Yn, int64_t n, int nz, const double* scales, void* y, hipStream_t s);
hipError_t launch_mr2(int ctype, const void* Pd, const void* Pl, const void* b, int64_t n, int nz, double* coef,
                      hipStream_t s);
hipError_t launch_mr2_combine(int ctype, const void* yd, const void* yl, const double* coef, void* y, int64_t n,
                              int nz, hipStream_t s);
}  // namespace ttn

struct ttn_sweep_src {
  const ttn_ttno* op = nullptr;
  const ttn_block* blk = nullptr;
  int n = 0;
  std::vector<int> tgt, src;          // host copies
  int32_t* d_tgt = nullptr;           // device [n]
  int32_t* d_src = nullptr;           // device [n]
  const double* coef = nullptr;       // device [n] (caller-owned)
  std::vector<std::vector<int>> rounds;  // term ids per round (unique targets)
  int32_t* d_perm = nullptr;          // device concatenation of rounds (term ids)
  int32_t* d_rtgt = nullptr;          // targets in round order
  int32_t* d_rsrc = nullptr;          // sources in round order
  double* d_rcoef = nullptr;          // coefficients in round order (gathered per step)
  ttn_envs* envs = nullptr;
  std::vector<void*> mem;
  int32_t* d_csr_ptr = nullptr;    // [k+1] terms of each target
  int32_t* d_csr_terms = nullptr;  // [n]
};

struct ttn_sweep {
  ttn_ctx* ctx = nullptr;
  const ttn_tree* t = nullptr;
  const ttn_ttno* op = nullptr;
  ttn_block* y = nullptr;
  ttn_dtype compute = TTN_F64;
  int ct = 0;
  int k = 0;
  std::vector<ttn_sweep_src> src;
  ttn_envs* henv = nullptr;
  std::vector<void*> hmem;
  int32_t* d_iota = nullptr;
  const double* shift = nullptr;
  // MINRES work: 7 vectors [k][n_loc_max] + state
  void* vec = nullptr;
  int64_t nmax = 0;
  MinresState* st = nullptr;
  int32_t* d_active = nullptr;  // number of MINRES states not yet converged (the contraction gate)
  // eager MINRES: reads of d_active land in a pinned ring, each followed by an event
  static constexpr int kRing = 4;
  int32_t* h_active = nullptr;
  hipEvent_t ev_active[kRing] = {};
  void* fit_scratch = nullptr;  // [max terms][n_loc_max] per-term local results
  // learned local map: candidate bookkeeping for 2k states (DIAG + MLP)
  int32_t* d_pair2 = nullptr;   // [2k] environment slot of each candidate (j mod k)
  double* d_shift2 = nullptr;   // [2k]
  double* d_coef = nullptr;     // [k][2] minimal-residual coefficients
  double* d_scales = nullptr;   // [k][2] (|b_j|, sigma_j)
  // sweep executor: Euler tour and captured graphs (one per option set)
  std::vector<int> tour;
  struct GraphRec {
    std::string key;
    hipGraphExec_t exec = nullptr;
    double flops = 0;  // algorithmic flops of one replay
  };
  std::vector<GraphRec> graphs;
  std::vector<std::string> warm;  // option sets already run eagerly (plans and tables built)
  ~ttn_sweep() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    (void)hipFree(fit_scratch);
    (void)hipFree(d_pair2);
    (void)hipFree(d_shift2);
    (void)hipFree(d_coef);
    (void)hipFree(d_scales);
    for (auto& s : src) {
      for (void* p : s.mem) (void)hipFree(p);
      (void)hipFree(s.d_tgt);
      (void)hipFree(s.d_src);
      (void)hipFree(s.d_perm);
      (void)hipFree(s.d_rtgt);
      (void)hipFree(s.d_rsrc);
      (void)hipFree(s.d_rcoef);
      (void)hipFree(s.d_csr_ptr);
      (void)hipFree(s.d_csr_terms);
      delete s.envs;
    }
    for (void* p : hmem) (void)hipFree(p);
    delete henv;
    (void)hipFree(d_iota);
    (void)hipFree(vec);
    (void)hipFree(st);
    (void)hipFree(d_active);
    if (h_active) (void)hipHostFree(h_active);
    for (hipEvent_t e : ev_active)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

template <typename T>
bool dmalloc(T** p, size_t bytes) {
  return dev_malloc((void**)p, bytes);
}

// environment set for (bra = target block, ket = other) with op (nullable)
ttn_envs* make_envs(const ttn_tree* t, const ttn_block* bra, const ttn_ttno* op, const ttn_block* ket, int n_slots,
                    ttn_dtype dt, std::vector<void*>& mem, bool& ok) {
  ttn_envs* e = new ttn_envs();
  e->t = t;
  e->n_slots = n_slots;
  e->Db = bra->D;
  e->Da = ket->D;
  e->identity = op == nullptr;
  e->M = op ? op->M : std::vector<int>(t->n, 1);
  e->dt = dt;
  e->slot.assign(2 * t->n, nullptr);
  const size_t es = dt == TTN_F64 ? 8 : 4;
  ok = true;
  for (int u = 0; u < t->n; ++u) {
    if (u == t->root) continue;
    const size_t bytes = (size_t)n_slots * e->Db[u] * e->M[u] * e->Da[u] * es;
    for (int s = 0; s < 2; ++s) {
      void* p = nullptr;
      if (!dev_malloc(&p, bytes)) {
        ok = false;
        return e;
      }
      mem.push_back(p);
      e->slot[2 * u + s] = p;
    }
  }
  return e;
}

#define HIPCHK(ctx, e)                                                                 \
  do {                                                                                 \
    hipError_t _e = (e);                                                               \
    if (_e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(_e));   \
  } while (0)

bool als_shape(const ttn_sweep* sw) {
  return sw->henv && sw->src.size() == 1 && sw->src[0].op == nullptr && sw->src[0].n == sw->k;
}

// local right-hand sides b_j = <y_j-environment | phi_s(j)> at node u (identity environments)
ttn_status local_rhs(ttn_sweep* sw, int u, void* b) {
  auto& s = sw->src[0];
  return heff_apply_rows(sw->ctx, sw->t, nullptr, s.envs, u, sw->k, nullptr, s.d_src, nullptr, sw->k, nullptr, nullptr,
                         s.blk->ptr[u], s.blk->k, b, TTN_HEFF_NO_SHIFT, sw->compute);
}

// diag(H_eff) - s_j at node u
ttn_status local_diag(ttn_sweep* sw, int u, void* dg) {
  return heff_apply_block(sw->ctx, sw->t, sw->op, sw->henv, u, sw->k, nullptr, nullptr, sw->shift, nullptr, nullptr, 0,
                          dg, TTN_HEFF_DIAG, sw->compute == TTN_BF16 ? TTN_F32 : sw->compute);
}

// LEARNED local step: y_D = b / d, y_L = MLP tiles, y_u = a y_D + c y_L with
// (a, c) minimising the local residual of the shifted system.
ttn_status learned_step(ttn_sweep* sw, int u, const ttn_solve_opts* opts, void* b, void* dg, void* cand, void* img,
                        void* out) {
  ttn_ctx* ctx = sw->ctx;
  const int k = sw->k, ct = sw->ct;
  const int64_t n = sw->y->size[u];
  const size_t es = ct == 0 ? 8 : 4;
  if (!opts->mlp_params) return api_fail(ctx, TTN_E_ARG, "LEARNED needs MLP parameters");
  if (opts->mlp_compute != TTN_BF16 && opts->mlp_compute != TTN_F32)
    return api_fail(ctx, TTN_E_DTYPE, "MLP computes in BF16 or FP32");
  void* yD = cand;
  void* yL = (char*)cand + (size_t)k * n * es;
  HIPCHK(ctx, launch_diag_solve(ct, b, dg, yD, n * k, ctx->stream));
  // network inference in groups of states that fit the workspace:
  // per tile row 4x256 activations + 128 features + 64 outputs (FP32)
  const int64_t ntiles = (n + 63) / 64;
  const int64_t row_bytes = (4 * 256 + 128 + 64) * 4;
  const int64_t cap_rows = std::min<int64_t>((int64_t)(ctx->ws_bytes / row_bytes), INT32_MAX / 1024);
  if (cap_rows < ntiles) return api_fail(ctx, TTN_E_WORKSPACE, "workspace too small for the learned preconditioner");
  const int g = (int)std::max<int64_t>(1, std::min<int64_t>(k, cap_rows / ntiles));
  ctx->ws_last_plan = nullptr;
  float* acts = (float*)ctx->ws;
  for (int z0 = 0; z0 < k; z0 += g) {
    const int gz = std::min(g, k - z0);
    const int64_t rows = ntiles * gz;
    float* X = acts + rows * 1024;
    float* Yn = X + rows * 128;
    HIPCHK(ctx, launch_features(ct, (const char*)b + (size_t)z0 * n * es, (const char*)dg + (size_t)z0 * n * es, n, gz,
                                sw->d_scales + 2 * z0, X, ctx->stream));
    ttn_status r = ttn_mlp_forward(ctx, opts->mlp_params, (int32_t)rows, X, Yn, acts, (ttn_dtype)opts->mlp_compute);
    if (r != TTN_OK) return r;
    HIPCHK(ctx, launch_untile(ct, Yn, n, gz, sw->d_scales + 2 * z0, (char*)yL + (size_t)z0 * n * es, ctx->stream));
  }
  // images of both candidates in one batched H_eff launch over 2k states
  const double* sh2 = nullptr;
  if (sw->shift) {
    HIPCHK(ctx, launch_gather_coef(sw->shift, sw->d_pair2, 2 * k, sw->d_shift2, ctx->stream));
    sh2 = sw->d_shift2;
  }
  ttn_status r = heff_apply_block(ctx, sw->t, sw->op, sw->henv, u, 2 * k, sw->d_pair2, nullptr, sh2, nullptr, cand,
                                  2 * k, img, TTN_HEFF_APPLY, sw->compute);
  if (r != TTN_OK) return r;
  HIPCHK(ctx, launch_mr2(ct, img, (char*)img + (size_t)k * n * es, b, n, k, sw->d_coef, ctx->stream));
  HIPCHK(ctx, launch_mr2_combine(ct, yD, yL, sw->d_coef, out, n, k, ctx->stream));
  if (opts->learned_coef &&
      hipMemcpyAsync(opts->learned_coef, sw->d_coef, (size_t)2 * k * 8, hipMemcpyDeviceToDevice, ctx->stream) !=
          hipSuccess)
    return api_fail(ctx, TTN_E_DEVICE, "copy of the combination coefficients failed");
  return TTN_OK;
}

ttn_status update_envs_across(ttn_sweep* sw, int u, int v) {
  ttn_ctx* ctx = sw->ctx;
  if (sw->henv) {
    ttn_status r = ttno_env_update(ctx, sw->t, sw->op, sw->y, sw->y, sw->k, sw->d_iota, sw->d_iota, u, v, sw->henv,
                                   sw->compute);
    if (r != TTN_OK) return r;
  }
  for (auto& s : sw->src) {
    ttn_status r = ttno_env_update(ctx, sw->t, s.op, sw->y, s.blk, s.n, s.d_tgt, s.d_src, u, v, s.envs, sw->compute);
    if (r != TTN_OK) return r;
  }
  return TTN_OK;
}

}  // namespace

extern "C" {

ttn_status ttn_sweep_create(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, ttn_block* target, int32_t n_src,
                            const ttn_ttno* const* src_op, const ttn_block* const* src_block, const int32_t* n_terms,
                            const int32_t* const* term_target, const int32_t* const* term_source,
                            const double* const* term_coef, const double* shift, ttn_dtype compute, ttn_sweep** out) {
  if (!ctx || !t || !target || !out || n_src < 0 || n_src > 2 || (n_src > 0 && (!src_block || !n_terms)))
    return api_fail(ctx, TTN_E_ARG, "bad sweep arguments");
  if (target->t != t) return api_fail(ctx, TTN_E_ARG, "tree mismatch");
  // FP64 storage with FP64 or FP32 matrix-core arithmetic; FP32 storage with
  // FP32 or BF16 arithmetic
  const bool f64 = compute == TTN_F64 || compute == TTN_F64_F32;
  if ((f64 && target->dt != TTN_F64) || (!f64 && target->dt != TTN_F32))
    return api_fail(ctx, TTN_E_DTYPE, "target dtype does not match the compute dtype");
  ttn_sweep* sw = new (std::nothrow) ttn_sweep();
  if (!sw) return api_fail(ctx, TTN_E_ARG, "out of host memory");
  sw->ctx = ctx;
  sw->t = t;
  sw->op = op;
  sw->y = target;
  sw->compute = compute;
  sw->ct = f64 ? 0 : 1;
  sw->k = target->k;
  sw->shift = shift;
  const size_t es = f64 ? 8 : 4;
  bool ok = true;
  std::vector<int32_t> iota(sw->k);
  for (int i = 0; i < sw->k; ++i) iota[i] = i;
  if (!dmalloc(&sw->d_iota, iota.size() * 4) ||
      !upload_sync(sw->d_iota, iota.data(), iota.size() * 4, ctx->stream)) {
    delete sw;
    return api_fail(ctx, TTN_E_DEVICE, "allocation failed");
  }
  if (op) {
    if (op->t != t) {
      delete sw;
      return api_fail(ctx, TTN_E_ARG, "tree mismatch");
    }
    sw->henv = make_envs(t, target, op, target, sw->k, target->dt, sw->hmem, ok);
    if (!ok) {
      delete sw;
      return api_fail(ctx, TTN_E_DEVICE, "environment allocation failed");
    }
  }
  for (int i = 0; i < n_src; ++i) {
    ttn_sweep_src s;
    s.op = src_op ? src_op[i] : nullptr;
    s.blk = src_block[i];
    s.n = n_terms[i];
    if (!s.blk || s.blk->t != t || s.n < 1 || !term_target || !term_source || !term_target[i] || !term_source[i]) {
      delete sw;
      return api_fail(ctx, TTN_E_ARG, "bad source term list");
    }
    if (s.blk->dt != target->dt) {
      delete sw;
      return api_fail(ctx, TTN_E_DTYPE, "source dtype differs from the target");
    }
    s.tgt.assign(term_target[i], term_target[i] + s.n);
    s.src.assign(term_source[i], term_source[i] + s.n);
    for (int j = 0; j < s.n; ++j)
      if (s.tgt[j] < 0 || s.tgt[j] >= sw->k || s.src[j] < 0 || s.src[j] >= s.blk->k) {
        delete sw;
        return api_fail(ctx, TTN_E_ARG, "term target/source out of range");
      }
    s.coef = term_coef ? term_coef[i] : nullptr;
    // rounds with unique targets (greedy)
    std::vector<std::vector<char>> used;
    for (int j = 0; j < s.n; ++j) {
      size_t r = 0;
      while (r < s.rounds.size() && used[r][s.tgt[j]]) ++r;
      if (r == s.rounds.size()) {
        s.rounds.push_back({});
        used.push_back(std::vector<char>(sw->k, 0));
      }
      s.rounds[r].push_back(j);
      used[r][s.tgt[j]] = 1;
    }
    std::vector<int32_t> perm, rt, rs;
    for (auto& r : s.rounds)
      for (int j : r) {
        perm.push_back(j);
        rt.push_back(s.tgt[j]);
        rs.push_back(s.src[j]);
      }
    const size_t nb = (size_t)s.n * 4;
    if (!dmalloc(&s.d_tgt, nb) || !dmalloc(&s.d_src, nb) || !dmalloc(&s.d_perm, nb) || !dmalloc(&s.d_rtgt, nb) ||
        !dmalloc(&s.d_rsrc, nb) || !dmalloc(&s.d_rcoef, (size_t)s.n * 8) ||
        !upload_sync(s.d_tgt, s.tgt.data(), nb, ctx->stream) ||
        !upload_sync(s.d_src, s.src.data(), nb, ctx->stream) ||
        !upload_sync(s.d_perm, perm.data(), nb, ctx->stream) ||
        !upload_sync(s.d_rtgt, rt.data(), nb, ctx->stream) ||
        !upload_sync(s.d_rsrc, rs.data(), nb, ctx->stream)) {
      sw->src.push_back(s);
      delete sw;
      return api_fail(ctx, TTN_E_DEVICE, "allocation failed");
    }
    {
      std::vector<int32_t> ptr(sw->k + 1, 0), terms;
      for (int j = 0; j < s.n; ++j) ptr[s.tgt[j] + 1]++;
      for (int i = 0; i < sw->k; ++i) ptr[i + 1] += ptr[i];
      terms.assign(s.n, 0);
      std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
      for (int j = 0; j < s.n; ++j) terms[fill[s.tgt[j]]++] = j;
      if (!dmalloc(&s.d_csr_ptr, ptr.size() * 4) || !dmalloc(&s.d_csr_terms, (size_t)s.n * 4) ||
          !upload_sync(s.d_csr_ptr, ptr.data(), ptr.size() * 4, ctx->stream) ||
          !upload_sync(s.d_csr_terms, terms.data(), (size_t)s.n * 4, ctx->stream)) {
        sw->src.push_back(s);
        delete sw;
        return api_fail(ctx, TTN_E_DEVICE, "allocation failed");
      }
    }
    s.envs = make_envs(t, target, s.op, s.blk, s.n, target->dt, s.mem, ok);
    sw->src.push_back(s);
    if (!ok) {
      delete sw;
      return api_fail(ctx, TTN_E_DEVICE, "environment allocation failed");
    }
  }
  // MINRES work vectors
  int64_t nmax = 1;
  for (int u = 0; u < t->n; ++u) nmax = std::max(nmax, target->size[u]);
  sw->nmax = nmax;
  int max_terms = 0;
  for (auto& s : sw->src) max_terms = std::max(max_terms, s.n);
  if (!dmalloc(&sw->vec, (size_t)8 * sw->k * nmax * es) || !dmalloc(&sw->st, (size_t)sw->k * sizeof(MinresState)) ||
      !dmalloc(&sw->d_active, 16) || !dmalloc(&sw->fit_scratch, (size_t)max_terms * nmax * es) ||
      !pinned_malloc((void**)&sw->h_active, ttn_sweep::kRing * sizeof(int32_t))) {
    delete sw;
    return api_fail(ctx, TTN_E_DEVICE, "allocation failed");
  }
  for (hipEvent_t& e : sw->ev_active)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      delete sw;
      return api_fail(ctx, TTN_E_DEVICE, "hipEventCreate failed");
    }
  {
    std::vector<int32_t> pair2(2 * sw->k);
    for (int i = 0; i < 2 * sw->k; ++i) pair2[i] = i % sw->k;
    if (!dmalloc(&sw->d_pair2, pair2.size() * 4) || !dmalloc(&sw->d_shift2, (size_t)2 * sw->k * 8) ||
        !dmalloc(&sw->d_coef, (size_t)2 * sw->k * 8) || !dmalloc(&sw->d_scales, (size_t)2 * sw->k * 8) ||
        !upload_sync(sw->d_pair2, pair2.data(), pair2.size() * 4, ctx->stream)) {
      delete sw;
      return api_fail(ctx, TTN_E_DEVICE, "allocation failed");
    }
  }
  *out = sw;
  return TTN_OK;
}

ttn_status ttn_sweep_run(ttn_ctx* ctx, ttn_sweep* sw, const ttn_solve_opts* opts, int32_t n_sweeps,
                         int32_t init_first, int32_t use_graph, int32_t* iters_out, double* resid_out) {
  if (!ctx || !sw || !opts || sw->ctx != ctx || n_sweeps < 0) return api_fail(ctx, TTN_E_ARG, "bad sweep arguments");
  const ttn_tree* t = sw->t;
  if (sw->tour.empty()) {
    // depth-first Euler tour from the root, children in index order
    std::vector<std::pair<int, size_t>> stk{{t->root, 0}};
    sw->tour.push_back(t->root);
    while (!stk.empty()) {
      auto& top = stk.back();
      const int u = top.first;
      if (top.second < t->ch[u].size()) {
        const int c = t->ch[u][top.second++];
        sw->tour.push_back(c);
        stk.push_back({c, 0});
      } else {
        stk.pop_back();
        if (!stk.empty()) sw->tour.push_back(stk.back().first);
      }
    }
  }
  auto run = [&]() -> ttn_status {
    if (init_first) {
      ttn_status r = ttn_sweep_init(sw, t->root);
      if (r != TTN_OK) return r;
    }
    ttn_solve_opts skip = *opts;
    skip.mode = TTN_SOLVE_SKIP;
    std::vector<char> seen(t->n);
    for (int s = 0; s < n_sweeps; ++s) {
      std::fill(seen.begin(), seen.end(), 0);
      for (size_t i = 0; i < sw->tour.size(); ++i) {
        const int u = sw->tour[i];
        const int nxt = i + 1 < sw->tour.size() ? sw->tour[i + 1] : -1;
        const ttn_solve_opts* o = seen[u] ? &skip : opts;
        seen[u] = 1;
        ttn_status r = sweep_step(ctx, sw, u, nxt, o, iters_out, resid_out);
        if (r != TTN_OK) return r;
      }
    }
    return TTN_OK;
  };
  // graphs: not under profiling (events), not on the legacy null stream, and
  // not for MINRES runs long enough to take host-side convergence checks
  const bool capturable = use_graph && !ctx->profile && ctx->stream != nullptr;
  if (!capturable) return run();
  std::ostringstream key;
  key << opts->mode << ":" << opts->maxiter << ":" << opts->rtol << ":" << (const void*)opts->mlp_params << ":"
      << opts->mlp_compute << ":" << (const void*)opts->learned_coef << ":" << opts->refine << ":" << opts->warm << ":"
      << opts->precond << ":" << opts->precond_damp << ":"
      << n_sweeps << ":" << init_first << ":"
      << (const void*)iters_out << ":" << (const void*)resid_out;
  const std::string k = key.str();
  for (auto& g : sw->graphs)
    if (g.key == k) {
      if (hipGraphLaunch(g.exec, ctx->stream) != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, "graph launch failed");
      ctx->flops_done += g.flops;
      return TTN_OK;
    }
  if (std::find(sw->warm.begin(), sw->warm.end(), k) == sw->warm.end()) {
    // first run of this option set: eager, so that every plan, table and
    // workspace the sweep needs exists before a capture
    ttn_status r = run();
    if (r == TTN_OK) sw->warm.push_back(k);
    return r;
  }
  const double f0 = ctx->flops_done;
  if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return api_fail(ctx, TTN_E_DEVICE, "stream capture could not start");
  ttn_status r = run();
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(ctx->stream, &graph);
  if (r != TTN_OK || ec != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    ctx->flops_done = f0;
    return r != TTN_OK ? r : api_fail(ctx, TTN_E_DEVICE, "stream capture failed");
  }
  ttn_sweep::GraphRec rec;
  rec.key = k;
  rec.flops = ctx->flops_done - f0;
  const hipError_t ei = hipGraphInstantiate(&rec.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    ctx->flops_done = f0;
    return api_fail(ctx, TTN_E_DEVICE, "graph instantiation failed");
  }
  sw->graphs.push_back(rec);
  // the capture recorded the work without running it: run it now
  if (hipGraphLaunch(rec.exec, ctx->stream) != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, "graph launch failed");
  return TTN_OK;
}

ttn_status ttn_sweep_harvest(ttn_ctx* ctx, ttn_sweep* sw, int32_t node, float* X, float* T, double* scales) {
  if (!ctx || !sw || sw->ctx != ctx || !X || !T || !scales) return api_fail(ctx, TTN_E_ARG, "bad harvest arguments");
  if (node < 0 || node >= sw->t->n) return api_fail(ctx, TTN_E_ARG, "bad node");
  if (!als_shape(sw)) return api_fail(ctx, TTN_E_ARG, "harvest needs an ALS sweep");
  const int k = sw->k;
  const size_t es = sw->ct == 0 ? 8 : 4;
  const int64_t n = sw->y->size[node];
  void* b = sw->vec;
  void* dg = (char*)sw->vec + (size_t)k * sw->nmax * es;
  ttn_status r = local_rhs(sw, node, b);
  if (r != TTN_OK) return r;
  r = local_diag(sw, node, dg);
  if (r != TTN_OK) return r;
  HIPCHK(ctx, launch_features(sw->ct, b, dg, n, k, scales, X, ctx->stream));
  HIPCHK(ctx, launch_targets(sw->ct, sw->y->ptr[node], b, dg, n, k, scales, T, ctx->stream));
  return TTN_OK;
}

ttn_status ttn_sweep_destroy(ttn_sweep* sw) {
  if (sw) (void)hipStreamSynchronize(sw->ctx->stream);
  delete sw;
  return TTN_OK;
}

ttn_status ttn_sweep_init(ttn_sweep* sw, int32_t centre) {
  if (!sw || centre < 0 || centre >= sw->t->n) return api_fail(sw ? sw->ctx : nullptr, TTN_E_ARG, "bad centre");
  const ttn_tree* t = sw->t;
  // post-order of the tree rooted at `centre`: every edge toward the centre
  std::vector<std::pair<int, int>> order;
  std::vector<std::pair<int, int>> stk{{centre, -1}};
  std::vector<std::pair<int, int>> visit;
  while (!stk.empty()) {
    auto [u, frm] = stk.back();
    stk.pop_back();
    visit.push_back({u, frm});
    for (int w : t->nb[u])
      if (w != frm) stk.push_back({w, u});
  }
  for (auto it = visit.rbegin(); it != visit.rend(); ++it)
    if (it->second >= 0) order.push_back(*it);
  for (auto& e : order) {
    ttn_status r = update_envs_across(sw, e.first, e.second);
    if (r != TTN_OK) return r;
  }
  return TTN_OK;
}

ttn_status sweep_step(ttn_ctx* ctx, ttn_sweep* sw, int32_t node, int32_t next, const ttn_solve_opts* opts,
                      int32_t* iters_out, double* resid_out) {
  if (!ctx || !sw || !opts || sw->ctx != ctx) return api_fail(ctx, TTN_E_ARG, "bad arguments");
  const ttn_tree* t = sw->t;
  if (node < 0 || node >= t->n || (next >= 0 && t->leg_of(node, next) < 0))
    return api_fail(ctx, TTN_E_ARG, "next is not a neighbour of node");
  const int u = node, k = sw->k, ct = sw->ct;
  const size_t es = ct == 0 ? 8 : 4;
  const int64_t n = sw->y->size[u];
  char* base = (char*)sw->vec;
  auto vbuf = [&](int i) { return (void*)(base + (size_t)i * k * sw->nmax * es); };
  void* y_u = sw->y->ptr[u];
  ttn_status r = TTN_OK;
  const int mode = opts->mode;
  if (mode == TTN_SOLVE_MINRES || mode == TTN_SOLVE_DIAG || mode == TTN_SOLVE_LEARNED) {
    if (!als_shape(sw))
      return api_fail(ctx, TTN_E_ARG, "ALS sweep needs an operator and one identity source term per state");
    // local right-hand side b_j = (y_j, phi_s(j)) identity environment contracted with phi_u
    void* b = vbuf(0);
    r = local_rhs(sw, u, b);
    if (r != TTN_OK) return r;
    if (mode == TTN_SOLVE_DIAG || mode == TTN_SOLVE_LEARNED) {
      void* dg = vbuf(1);
      r = local_diag(sw, u, dg);
      if (r != TTN_OK) return r;
      if (mode == TTN_SOLVE_DIAG) {
        hipError_t e = launch_diag_solve(ct, b, dg, y_u, n * k, ctx->stream);
        if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
      } else {
        // candidates [2k][n] span vbuf(2..3), their images vbuf(4..5)
        r = learned_step(sw, u, opts, b, dg, vbuf(2), vbuf(4), y_u);
        if (r != TTN_OK) return r;
      }
    } else {
      if (opts->maxiter < 0 || !(opts->rtol >= 0) || opts->refine < 0)
        return api_fail(ctx, TTN_E_ARG, "bad MINRES options");
      if (opts->refine > 0 && ct != 0)
        return api_fail(ctx, TTN_E_DTYPE, "mixed-precision refinement needs an FP64 sweep");
      if (opts->warm < TTN_WARM_NONE || opts->warm > TTN_WARM_LEARNED || (opts->warm != TTN_WARM_NONE && opts->refine > 0))
        return api_fail(ctx, TTN_E_ARG, "corrected MINRES start: warm 0..2, and only without refinement");
      const int pc = opts->precond;
      if (pc < TTN_PRECOND_NONE || pc > TTN_PRECOND_DAMPED_DIAG ||
          (pc != TTN_PRECOND_NONE && (opts->refine > 0 || opts->warm != TTN_WARM_NONE)) ||
          (pc == TTN_PRECOND_DAMPED_DIAG && !(opts->precond_damp >= 0)))
        return api_fail(ctx, TTN_E_ARG, "preconditioner: 0..2, with refine = 0 and warm = NONE, damping >= 0");
      void *v = vbuf(1), *vp = vbuf(2), *p = vbuf(3), *d1 = vbuf(4), *d2 = vbuf(5);
      void *dsq = vbuf(6), *tv = vbuf(7);  // preconditioner D^-1/2 and the scaled Krylov vector
      // batched MINRES on (H_eff - s) x = rhs, warm start x with Ax0 = (H_eff - s) x
      auto minres = [&](void* x, const void* rhs, const void* ax0, ttn_dtype comp, double rtol) -> ttn_status {
        hipError_t e = launch_minres_init(ct, rhs, ax0, v, vp, d1, d2, n, k, rtol, sw->st, sw->d_active, ctx->stream);
        if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
        void *vv = v, *vvp = vp, *dp = d1, *dpp = d2;
        // Every `seg` iterations a one-workgroup kernel counts the states not
        // yet converged into d_active; the iteration's contraction kernels read
        // it first and do nothing once it is zero, so the work stops on the
        // device without the host.  Eagerly, the count is also copied to a
        // pinned ring (no wait) and the host stops enqueueing once a completed
        // copy reads zero; it waits for the oldest copy only when it runs four
        // segments ahead of the device.  Under stream capture all maxiter
        // iterations are recorded and the gate alone ends the work.
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        const bool capturing =
            hipStreamIsCapturing(ctx->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
        const int seg = 25;
        int issued = 0, polled = 0;
        bool stop = false;
        struct GateGuard {
          ttn_ctx* c;
          ~GateGuard() {
            c->gate = nullptr;
            c->reuse_free = false;
          }
        } guard{ctx};
        const char* re = getenv("TTN_REUSE_FREE");
        const bool reuse_on = !(re && re[0] == '0');
        for (int it = 0; it < opts->maxiter && !stop; ++it) {
          // the environments are fixed during the solve: from the second
          // product on, the stages that do not involve the Krylov vector (the
          // operator-environment partials) are reused from the workspace
          const void* xin = vv;
          if (pc != TTN_PRECOND_NONE) {  // (D^-1/2 A D^-1/2) v: scale, apply, scale
            HIPCHK(ctx, launch_ew_mul(ct, dsq, vv, tv, n * k, sw->d_active, ctx->stream));
            xin = tv;
          }
          ctx->gate = sw->d_active;
          ctx->reuse_free = reuse_on && it > 0;
          ttn_status rr = heff_apply_block(ctx, t, sw->op, sw->henv, u, k, nullptr, nullptr, sw->shift, nullptr, xin, k,
                                           p, TTN_HEFF_APPLY, comp);
          ctx->gate = nullptr;
          ctx->reuse_free = false;
          if (rr != TTN_OK) return rr;
          if (pc != TTN_PRECOND_NONE) HIPCHK(ctx, launch_ew_mul(ct, dsq, p, p, n * k, sw->d_active, ctx->stream));
          e = launch_minres_step(ct, x, vv, vvp, p, dp, dpp, n, k, sw->st, ctx->stream);
          if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
          std::swap(vv, vvp);
          std::swap(dp, dpp);
          if ((it + 1) % seg == 0 && it + 1 < opts->maxiter) {
            e = launch_minres_count(sw->st, k, sw->d_active, ctx->stream);
            if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
            if (capturing) continue;
            const int R = ttn_sweep::kRing;
            if (issued - polled == R) {  // bounded run-ahead: wait for the oldest read
              if (hipEventSynchronize(sw->ev_active[polled % R]) != hipSuccess)
                return api_fail(ctx, TTN_E_DEVICE, "convergence read failed");
              stop = ((volatile int32_t*)sw->h_active)[polled % R] == 0;
              ++polled;
              if (stop) break;
            }
            if (hipMemcpyAsync(sw->h_active + issued % R, sw->d_active, 4, hipMemcpyDeviceToHost, ctx->stream) !=
                    hipSuccess ||
                hipEventRecord(sw->ev_active[issued % R], ctx->stream) != hipSuccess)
              return api_fail(ctx, TTN_E_DEVICE, "convergence read failed");
            ++issued;
            while (polled < issued && hipEventQuery(sw->ev_active[polled % R]) == hipSuccess) {
              stop = ((volatile int32_t*)sw->h_active)[polled % R] == 0;
              ++polled;
              if (stop) break;
            }
          }
        }
        return TTN_OK;
      };
      static const bool leaf_fused = !(getenv("TTN_LEAF_MINRES") && getenv("TTN_LEAF_MINRES")[0] == '0');
      const bool same_prec = (sw->compute == TTN_F64 && ct == 0) || (sw->compute == TTN_F32 && ct == 1);
      LeafHeffArgs la;
      if (leaf_fused && pc == TTN_PRECOND_NONE && opts->refine == 0 && opts->warm == TTN_WARM_NONE && same_prec &&
          n <= 256 && leaf_heff_fusable(ctx, t, sw->op, sw->henv, u, ct, la) && la.Da == la.Db &&
          (int64_t)la.Da * la.d == n && k <= sw->henv->n_slots) {
        // a leaf: warm-start product, initialisation and every iteration in
        // one launch (the H_eff products are recorded under the node's key)
        la.X = y_u;
        la.x_stride = n;
        la.x_rows = k;
        la.n_slots = k;
        la.Y = y_u;
        la.y_stride = n;
        la.y_rows = k;
        la.shift = sw->shift;
        la.n = k;
        la.flag = ctx->d_flag;
        const double Db = la.Db, Mw = la.M, Da = la.Da, d = la.d;
        const double per = 2.0 * (Db * Mw * Da * d + Db * d * Mw * d) * k * (opts->maxiter + 1.0);
        ctx->flops_done += per;
        const std::string key = "heff:" + std::to_string(u) + ":1:leafminres";
        ttn_prof_rec* pr = prof_begin(ctx, key.c_str(), "leaf_minres_kernel", per,
                                      (double)es * (k * (3.0 * n + Db * Mw * Da) + Mw * d * d), k);
        HIPCHK(ctx, launch_leaf_minres(ct, la, b, y_u, n, opts->rtol, opts->maxiter, sw->st, ctx->stream));
        prof_end(ctx, pr);
      } else if (opts->refine == 0 && opts->warm == TTN_WARM_NONE) {
        // p = (H_eff - s) y_u  (warm start)
        r = heff_apply_block(ctx, t, sw->op, sw->henv, u, k, nullptr, nullptr, sw->shift, nullptr, y_u, k, p,
                             TTN_HEFF_APPLY, sw->compute);
        if (r != TTN_OK) return r;
        if (pc != TTN_PRECOND_NONE) {
          // D^-1/2 from the local diagonal, then the scaled system: b <- D^-1/2 b,
          // z = D^1/2 y_u, its image D^-1/2 A y_u
          r = local_diag(sw, u, dsq);
          if (r != TTN_OK) return r;
          HIPCHK(ctx, launch_precond_scale(ct, dsq, dsq, n, k, pc, opts->precond_damp, ctx->stream));
          HIPCHK(ctx, launch_ew_mul(ct, dsq, p, p, n * k, nullptr, ctx->stream));
          HIPCHK(ctx, launch_ew_mul(ct, dsq, b, b, n * k, nullptr, ctx->stream));
          HIPCHK(ctx, launch_ew_div(ct, y_u, dsq, y_u, n * k, ctx->stream));
        }
        r = minres(y_u, b, p, sw->compute, opts->rtol);
        if (r != TTN_OK) return r;
        if (pc != TTN_PRECOND_NONE) HIPCHK(ctx, launch_ew_mul(ct, dsq, y_u, y_u, n * k, nullptr, ctx->stream));
      } else if (opts->refine == 0) {
        // corrected start: r0 = b - (H_eff - s) y_u, a minimal-residual DIAG
        // or learned correction c of r0, y_u += c, then MINRES from there
        void *ax = vbuf(6), *res = vbuf(7), *dg = vbuf(1), *cor = vbuf(2), *acor = vbuf(3);
        r = heff_apply_block(ctx, t, sw->op, sw->henv, u, k, nullptr, nullptr, sw->shift, nullptr, y_u, k, ax,
                             TTN_HEFF_APPLY, sw->compute);
        if (r != TTN_OK) return r;
        HIPCHK(ctx, launch_resid_zero(ct, b, ax, res, cor, n * k, ctx->stream));
        r = local_diag(sw, u, dg);
        if (r != TTN_OK) return r;
        if (opts->warm == TTN_WARM_DIAG) {
          HIPCHK(ctx, launch_diag_solve(ct, res, dg, cor, n * k, ctx->stream));
          r = heff_apply_block(ctx, t, sw->op, sw->henv, u, k, nullptr, nullptr, sw->shift, nullptr, cor, k, acor,
                               TTN_HEFF_APPLY, sw->compute);
          if (r != TTN_OK) return r;
          // best scale of the DIAG step (a 2x2 system with two equal images keeps c = 0)
          HIPCHK(ctx, launch_mr2(ct, acor, acor, res, n, k, sw->d_coef, ctx->stream));
          HIPCHK(ctx, launch_mr2_combine(ct, cor, cor, sw->d_coef, cor, n, k, ctx->stream));
          HIPCHK(ctx, launch_mr2_combine(ct, acor, acor, sw->d_coef, acor, n, k, ctx->stream));
        } else {
          // candidates [2k][n] packed from vbuf(2), their images packed from
          // vbuf(4) (the learned image starts k*n entries in); the correction
          // lands in vbuf(1), its image in vbuf(3)
          void* img = vbuf(4);
          r = learned_step(sw, u, opts, res, dg, vbuf(2), img, dg);
          if (r != TTN_OK) return r;
          cor = dg;
          HIPCHK(ctx, launch_mr2_combine(ct, img, (char*)img + (size_t)k * n * es, sw->d_coef, acor, n, k,
                                         ctx->stream));
        }
        HIPCHK(ctx, launch_axpy_rows(ct, cor, y_u, n * k, ctx->stream));
        HIPCHK(ctx, launch_axpy_rows(ct, acor, ax, n * k, ctx->stream));
        r = minres(y_u, b, ax, sw->compute, opts->rtol);
        if (r != TTN_OK) return r;
      } else {
        // iterative refinement: FP64 residual, correction by MINRES in FP32
        // matrix-core arithmetic on the FP64 tensors, FP64 update
        void *res = vbuf(6), *cor = vbuf(7);
        const double rtol_in = opts->rtol > 1e-6 ? opts->rtol : 1e-6;
        for (int step = 0; step < opts->refine; ++step) {
          r = heff_apply_block(ctx, t, sw->op, sw->henv, u, k, nullptr, nullptr, sw->shift, nullptr, y_u, k, p,
                               TTN_HEFF_APPLY, TTN_F64);
          if (r != TTN_OK) return r;
          hipError_t e = launch_resid_zero(ct, b, p, res, cor, n * k, ctx->stream);
          if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
          r = minres(cor, res, cor, TTN_F64_F32, rtol_in);
          if (r != TTN_OK) return r;
          e = launch_axpy_rows(ct, cor, y_u, n * k, ctx->stream);
          if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
        }
      }
      if (iters_out || resid_out) {
        hipError_t e = launch_minres_report(sw->st, k, iters_out, resid_out, nullptr, ctx->stream);
        if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
      }
    }
  } else if (mode == TTN_SOLVE_FIT) {
    // every term's local contribution (H_eff-type product with the (target,
    // source) environments) in one batched launch, then a segmented sum per
    // target: y_t = sum_{terms of t} c * scratch_term
    for (size_t si = 0; si < sw->src.size(); ++si) {
      auto& s = sw->src[si];
      if (!s.coef) return api_fail(ctx, TTN_E_ARG, "FIT needs coefficients");
      r = heff_apply_rows(ctx, t, s.op, s.envs, u, s.n, nullptr, s.d_src, nullptr, s.n, nullptr, nullptr,
                          s.blk->ptr[u], s.blk->k, sw->fit_scratch, TTN_HEFF_NO_SHIFT, sw->compute);
      if (r != TTN_OK) return r;
      if (si == 0) {
        hipError_t e = launch_seg_sum(ct, sw->fit_scratch, s.d_csr_ptr, s.d_csr_terms, s.coef, y_u, n, k, false,
                                      ctx->stream);
        if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
      } else {
        // second source set: accumulate on top through a temporary target
        void* tmp = vbuf(0);
        hipError_t e = launch_seg_sum(ct, sw->fit_scratch, s.d_csr_ptr, s.d_csr_terms, s.coef, tmp, n, k, false,
                                      ctx->stream);
        if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
        e = launch_axpy_rows(ct, tmp, y_u, n * k, ctx->stream);
        if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
      }
    }
  } else if (mode != TTN_SOLVE_SKIP) {
    return api_fail(ctx, TTN_E_ARG, "unknown solve mode");
  }
  if (next >= 0) {
    r = ttn_block_move_centre(ctx, sw->y, u, next);
    if (r != TTN_OK) return r;
    r = update_envs_across(sw, u, next);
    if (r != TTN_OK) return r;
  }
  return TTN_OK;
}

}  // extern "C"
