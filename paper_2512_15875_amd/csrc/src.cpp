// C ABI: successive randomized compression (SRC) of the products y_j ~ H x_j
// for the k states of a block (Sec. II.C.1; Eq. matrix random compression,
// Fig. random tensor, Fig. src).  The random test matrix of every state is a
// Khatri-Rao product: column l is the product vector over the physical nodes
// of the rows l of the per-node matrices Omega^(u) ([chi][d_u], passed in), so
// every sketch is an environment of <omega_l| H |x_j> with a bond-one bra --
// the pair-batched environment engine with k * chi pairs.
//
// Per node, leaves to root: the local sketch Y_u (k * chi rows) is one H_eff
// product whose child legs read the compressed children's environments
// B_{c->u} = <y|H|x_j> and whose parent leg reads the sketch environment
// parent -> u; it is written straight into y's node buffer ([k][chi][n_loc]),
// where a Householder QR of each state's [n_loc x chi] block (diag(R) >= 0)
// leaves the orthonormal Q in place -- y's node tensor with its parent leg
// first.  A node whose local space has no more than chi dimensions keeps it
// whole (identity).  Then B_{u->parent} is updated, and at the root the
// remaining network is contracted directly (one H_eff product).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "internal.h"

using namespace ttn;

namespace ttn {
hipError_t launch_qr(int ctype, void* X, int64_t size, const int32_t* roff, int m, int n, int64_t cstride, double* work,
                     double* R, int nz, int* flag, hipStream_t s);
hipError_t launch_set_identity(int ctype, void* X, int n, int k, hipStream_t s);
hipError_t launch_expand_complete(int ctype, const void* Qx, int64_t qstride, const void* S, int64_t sstride, void* A,
                                  int64_t astride, void* Y, int64_t ystride, int D, int n, int grow, int m, int k,
                                  hipStream_t s);
}  // namespace ttn

// Bond expansion of a block (x -> y with larger bonds, y = x as states): the
// same sketch environments as SRC with n columns, then leaves to root per
// node: X_u (x_u with the children legs in y's bases, parent leg open) and its
// QR, the local sketch S_u of H x, the rank-revealing completion of [Q_x | S_u]
// (expand.hip), and the environments <y|x>, <y|H|x> across the edge; the root
// is x_root in the children's new bases.
struct ttn_expand {
  ttn_ctx* ctx = nullptr;
  const ttn_tree* t = nullptr;
  const ttn_ttno* op = nullptr;
  const ttn_block* x = nullptr;
  ttn_block* y = nullptr;
  int n = 0, k = 0;
  ttn_dtype compute = TTN_F64;
  ttn_block om;                     // the n sketch columns as bond-one states
  ttn_envs senv;                    // <omega_l|H|x_j>, every directed edge, k * n slots
  ttn_envs hav;                     // <y_j|H|x_j> toward the root, k slots
  ttn_envs bxv;                     // <y_j|x_j> toward the root, k slots (identity)
  ttn_envs idv;                     // delta_{ba} on every edge toward the root, 1 slot (identity)
  std::vector<void*> mem;
  void* ones = nullptr;
  void* xs = nullptr;               // [k][D_u][rest] local x, then its Q
  void* ss = nullptr;               // [k n][rest] local sketches
  void* aw = nullptr;               // [k][D_u + n][rest] completion work
  int64_t max_rest = 0, max_d = 0;
  int32_t *d_l = nullptr, *d_j = nullptr, *d_zero = nullptr, *d_iota = nullptr;
  std::vector<int> post;
  ~ttn_expand() {
    for (void* p : mem) (void)hipFree(p);
  }
};

struct ttn_src {
  ttn_ctx* ctx = nullptr;
  const ttn_tree* t = nullptr;
  const ttn_ttno* op = nullptr;
  const ttn_block* x = nullptr;
  ttn_block* y = nullptr;
  int chi = 0, k = 0;
  ttn_dtype compute = TTN_F64;
  ttn_block om;                     // the chi sketch columns as bond-one states (pointers set per apply)
  ttn_envs senv;                    // <omega_l|H|x_j> environments, every directed edge, k * chi slots
  ttn_envs benv;                    // <y_j|H|x_j> environments toward the root, k slots
  std::vector<void*> mem;
  void* ones = nullptr;             // chi ones: the sketch "tensor" of an auxiliary node
  int32_t* d_l = nullptr;           // [k chi] sketch column of item p = j chi + l
  int32_t* d_j = nullptr;           // [k chi] state of item p
  int32_t* d_iota = nullptr;        // [k]
  std::vector<int> post;            // post-order of the nodes
  ~ttn_src() {
    for (void* p : mem) (void)hipFree(p);
  }
};

namespace {

// bonds of the compressed state: edge (u, parent) keeps min(chi, rows of
// node u's local space), the rows being the product of its children's
// compressed bonds and its physical dimension
std::vector<int> src_bonds(const ttn_tree* t, int chi, std::vector<int>& post) {
  std::vector<int> b(t->n, 0);
  post.clear();
  std::vector<std::pair<int, int>> st{{t->root, 0}};
  while (!st.empty()) {
    auto [u, i] = st.back();
    if (i < (int)t->ch[u].size()) {
      st.back().second++;
      st.push_back({t->ch[u][i], 0});
    } else {
      st.pop_back();
      post.push_back(u);
    }
  }
  for (int u : post) {
    if (u == t->root) continue;
    int64_t rows = t->phys[u];
    for (int c : t->ch[u]) rows *= b[c];
    b[u] = (int)std::min<int64_t>(chi, rows);
  }
  return b;
}

template <typename H>
bool alloc(H* s, void** p, size_t bytes) {
  if (!dev_malloc(p, bytes)) return false;
  s->mem.push_back(*p);
  return true;
}

std::vector<int> post_order(const ttn_tree* t) {
  std::vector<int> post;
  (void)src_bonds(t, 1, post);
  return post;
}

}  // namespace

extern "C" {

ttn_status ttn_src_bonds(const ttn_tree* t, int32_t chi, int32_t* bonds_out) {
  if (!t || !bonds_out || chi < 1) return api_fail(nullptr, TTN_E_ARG, "bad arguments");
  std::vector<int> post;
  const std::vector<int> b = src_bonds(t, chi, post);
  for (int u = 0; u < t->n; ++u) bonds_out[u] = b[u];
  return TTN_OK;
}

ttn_status ttn_src_create(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_block* x, ttn_block* y,
                          int32_t chi, ttn_dtype compute, ttn_src** out) {
  if (!ctx || !t || !op || !x || !y || !out) return api_fail(ctx, TTN_E_ARG, "null argument");
  if (chi < 1 || chi > 512) return api_fail(ctx, TTN_E_ARG, "chi outside [1, 512]");
  if (x->t != t || y->t != t || op->t != t) return api_fail(ctx, TTN_E_ARG, "tree mismatch");
  if (x->k != y->k || x->k < 1) return api_fail(ctx, TTN_E_SHAPE, "x and y must hold the same k >= 1 states");
  if (x->dt != y->dt || op->dt != x->dt) return api_fail(ctx, TTN_E_DTYPE, "x, y and the operator share one dtype");
  if ((compute == TTN_F64) != (x->dt == TTN_F64) || compute == TTN_BF16 || compute == TTN_F64_F32)
    return api_fail(ctx, TTN_E_DTYPE, "compute: TTN_F64 for FP64 tensors, TTN_F32 for FP32 tensors");
  if (t->n < 2) return api_fail(ctx, TTN_E_SHAPE, "single-node tree");
  ttn_src* s = new (std::nothrow) ttn_src();
  if (!s) return api_fail(ctx, TTN_E_ARG, "out of host memory");
  s->ctx = ctx;
  s->t = t;
  s->op = op;
  s->x = x;
  s->y = y;
  s->chi = chi;
  s->k = x->k;
  s->compute = compute;
  const std::vector<int> yb = src_bonds(t, chi, s->post);
  for (int u = 0; u < t->n; ++u)
    if (u != t->root && y->D[u] != yb[u]) {
      delete s;
      return api_fail(ctx, TTN_E_SHAPE, "y's bonds differ from ttn_src_bonds(chi)");
    }
  const size_t es = x->dt == TTN_F64 ? 8 : 4;
  const int k = s->k, kc = k * chi;
  // the sketch block: chi bond-one states
  s->om.t = t;
  s->om.k = chi;
  s->om.D.assign(t->n, 1);
  s->om.dt = x->dt;
  s->om.ptr.assign(t->n, nullptr);
  s->om.size.assign(t->n, 0);
  for (int u = 0; u < t->n; ++u) s->om.size[u] = t->phys[u];
  // environments
  auto make = [&](ttn_envs& e, int n_slots, const std::vector<int>& Db, bool down) -> bool {
    e.t = t;
    e.n_slots = n_slots;
    e.Db = Db;
    e.Da = x->D;
    e.M = op->M;
    e.identity = false;
    e.dt = x->dt;
    e.slot.assign(2 * t->n, nullptr);
    for (int u = 0; u < t->n; ++u) {
      if (u == t->root) continue;
      const size_t bytes = (size_t)n_slots * e.Db[u] * e.M[u] * e.Da[u] * es;
      for (int d = 0; d < (down ? 2 : 1); ++d)
        if (!alloc(s, &e.slot[2 * u + d], bytes)) return false;
    }
    return true;
  };
  std::vector<int> ones_b(t->n, 1);
  std::vector<int32_t> hl(kc), hj(kc), hi(k);
  for (int p = 0; p < kc; ++p) {
    hl[p] = p % chi;
    hj[p] = p / chi;
  }
  for (int j = 0; j < k; ++j) hi[j] = j;
  std::vector<double> ones_d(chi, 1.0);
  std::vector<float> ones_f(chi, 1.0f);
  if (!make(s->senv, kc, ones_b, true) || !make(s->benv, k, y->D, false) || !alloc(s, &s->ones, (size_t)chi * es) ||
      !alloc(s, (void**)&s->d_l, (size_t)kc * 4) || !alloc(s, (void**)&s->d_j, (size_t)kc * 4) ||
      !alloc(s, (void**)&s->d_iota, (size_t)k * 4) ||
      !upload_sync(s->d_l, hl.data(), hl.size() * 4, ctx->stream) ||
      !upload_sync(s->d_j, hj.data(), hj.size() * 4, ctx->stream) ||
      !upload_sync(s->d_iota, hi.data(), hi.size() * 4, ctx->stream) ||
      !upload_sync(s->ones, es == 8 ? (const void*)ones_d.data() : (const void*)ones_f.data(), (size_t)chi * es,
                   ctx->stream)) {
    delete s;
    return api_fail(ctx, TTN_E_DEVICE, "allocation failed");
  }
  *out = s;
  return TTN_OK;
}

ttn_status ttn_src_destroy(ttn_src* s) {
  if (s) (void)hipStreamSynchronize(s->ctx->stream);
  delete s;
  return TTN_OK;
}

ttn_status ttn_src_apply(ttn_ctx* ctx, ttn_src* s, const void* const* omega) {
  if (!ctx || !s || !omega || s->ctx != ctx) return api_fail(ctx, TTN_E_ARG, "bad arguments");
  const ttn_tree* t = s->t;
  const int k = s->k, chi = s->chi, kc = k * chi;
  const int ct = s->x->dt == TTN_F64 ? 0 : 1;
  for (int u = 0; u < t->n; ++u) {
    if (t->phys[u] > 1 && !omega[u]) return api_fail(ctx, TTN_E_ARG, "missing test matrix at a physical node");
    s->om.ptr[u] = t->phys[u] > 1 ? const_cast<void*>(omega[u]) : s->ones;
  }
  ttn_status r = TTN_OK;
  // 1. sketch environments <omega_l|H|x_j> on every edge: toward the root,
  //    then away from it (items p = j chi + l)
  for (int u : s->post)
    if (u != t->root) {
      r = ttno_env_update(ctx, t, s->op, &s->om, s->x, kc, s->d_l, s->d_j, u, t->parent[u], &s->senv, s->compute);
      if (r != TTN_OK) return r;
    }
  for (auto it = s->post.rbegin(); it != s->post.rend(); ++it)
    for (int c : t->ch[*it]) {
      r = ttno_env_update(ctx, t, s->op, &s->om, s->x, kc, s->d_l, s->d_j, *it, c, &s->senv, s->compute);
      if (r != TTN_OK) return r;
    }
  // 2.-4. leaves to root
  for (int u : s->post) {
    const int p = t->parent[u];
    if (p < 0) {
      // the root: everything left, contracted directly
      r = heff_apply_block(ctx, t, s->op, &s->benv, u, k, nullptr, nullptr, nullptr, nullptr, s->x->ptr[u], k,
                           s->y->ptr[u], TTN_HEFF_NO_SHIFT, s->compute);
      if (r != TTN_OK) return r;
      continue;
    }
    int64_t rows = t->phys[u];
    for (int c : t->ch[u]) rows *= s->y->D[c];
    if (rows <= chi) {
      // the whole local space is kept
      hipError_t e = launch_set_identity(ct, s->y->ptr[u], (int)rows, k, ctx->stream);
      if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
    } else {
      // local sketch Y[j chi + l] into y's node buffer: child legs read the
      // compressed children's environments (slot j), the parent leg the
      // sketch environment parent -> u (slot j chi + l)
      ttn_envs mix;
      mix.t = t;
      mix.n_slots = kc;
      mix.Db = s->y->D;
      mix.Db[u] = 1;
      mix.Da = s->x->D;
      mix.M = s->op->M;
      mix.dt = s->x->dt;
      mix.slot.assign(2 * t->n, nullptr);
      mix.slot[ttn_envs::dslot(t, p, u)] = s->senv.slot[ttn_envs::dslot(t, p, u)];
      ctx->leg_tabs.clear();
      for (int c : t->nb[u]) {
        if (c == p) {
          ctx->leg_tabs.push_back({nullptr, kc});
        } else {
          mix.slot[ttn_envs::dslot(t, c, u)] = s->benv.slot[ttn_envs::dslot(t, c, u)];
          ctx->leg_tabs.push_back({s->d_j, k});
        }
      }
      r = ttn::heff_apply_rows(ctx, t, s->op, &mix, u, kc, nullptr, s->d_j, nullptr, kc, nullptr, nullptr,
                               s->x->ptr[u], k, s->y->ptr[u], TTN_HEFF_NO_SHIFT, s->compute);
      ctx->leg_tabs.clear();
      if (r != TTN_OK) return r;
      // Householder QR of each state's [rows x chi] block, Q left in place
      const std::vector<int> dims = s->y->legdims(u);
      int64_t cs = 0;
      int m = 0;
      ttn_status code = TTN_OK;
      const int32_t* ro = leg_rows_table(ctx, dims, 0, cs, m, code);
      if (!ro) return code;
      const size_t work = (size_t)k * 2 * m * chi * sizeof(double);
      const size_t rbytes = (size_t)k * (chi * chi + chi) * sizeof(double);
      auto al = [](size_t v) { return (v + 255) / 256 * 256; };
      if (al(work) + al(rbytes) > ctx->ws_bytes) return api_fail(ctx, TTN_E_WORKSPACE, "workspace too small for QR");
      ctx->ws_last_plan = nullptr;
      double* wk = (double*)ctx->ws;
      double* R = (double*)((char*)ctx->ws + al(work));
      hipError_t e = launch_qr(ct, s->y->ptr[u], s->y->size[u], ro, m, chi, cs, wk, R, k, ctx->d_flag, ctx->stream);
      if (e != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(e));
    }
    // B_{u -> parent} = <y_j| H |x_j>
    r = ttno_env_update(ctx, t, s->op, s->y, s->x, k, s->d_iota, s->d_iota, u, p, &s->benv, s->compute);
    if (r != TTN_OK) return r;
  }
  return TTN_OK;
}


ttn_status ttn_expand_create(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_block* x, ttn_block* y,
                             int32_t n_sketch, ttn_dtype compute, ttn_expand** out) {
  if (!ctx || !t || !op || !x || !y || !out) return api_fail(ctx, TTN_E_ARG, "null argument");
  if (n_sketch < 1 || n_sketch > 128) return api_fail(ctx, TTN_E_ARG, "n_sketch outside [1, 128]");
  if (x->t != t || y->t != t || op->t != t) return api_fail(ctx, TTN_E_ARG, "tree mismatch");
  if (x->k != y->k || x->k < 1) return api_fail(ctx, TTN_E_SHAPE, "x and y must hold the same k >= 1 states");
  if (x->dt != y->dt || op->dt != x->dt) return api_fail(ctx, TTN_E_DTYPE, "x, y and the operator share one dtype");
  if ((compute == TTN_F64) != (x->dt == TTN_F64) || compute == TTN_BF16 || compute == TTN_F64_F32)
    return api_fail(ctx, TTN_E_DTYPE, "compute: TTN_F64 for FP64 tensors, TTN_F32 for FP32 tensors");
  if (t->n < 2) return api_fail(ctx, TTN_E_SHAPE, "single-node tree");
  ttn_expand* e = new (std::nothrow) ttn_expand();
  if (!e) return api_fail(ctx, TTN_E_ARG, "out of host memory");
  e->ctx = ctx;
  e->t = t;
  e->op = op;
  e->x = x;
  e->y = y;
  e->n = n_sketch;
  e->k = x->k;
  e->compute = compute;
  e->post = post_order(t);
  for (int u = 0; u < t->n; ++u) {
    if (u == t->root) continue;
    int64_t rest = t->phys[u];
    for (int c : t->ch[u]) rest *= y->D[c];
    const int grow = y->D[u] - x->D[u];
    if (grow < 0 || grow > n_sketch || y->D[u] > rest || x->D[u] + n_sketch > 256) {
      delete e;
      return api_fail(ctx, TTN_E_SHAPE,
                      "each bond of y must lie in [x's bond, x's bond + n_sketch] and within its node's local space "
                      "(x's bond + n_sketch <= 256)");
    }
    e->max_rest = std::max(e->max_rest, rest);
    e->max_d = std::max<int64_t>(e->max_d, x->D[u]);
  }
  const size_t es = x->dt == TTN_F64 ? 8 : 4;
  const int k = e->k, kn = k * n_sketch;
  e->om.t = t;
  e->om.k = n_sketch;
  e->om.D.assign(t->n, 1);
  e->om.dt = x->dt;
  e->om.ptr.assign(t->n, nullptr);
  e->om.size.assign(t->n, 0);
  for (int u = 0; u < t->n; ++u) e->om.size[u] = t->phys[u];
  auto make = [&](ttn_envs& v, int n_slots, const std::vector<int>& Db, const std::vector<int>& Da, bool ident,
                  bool down) -> bool {
    v.t = t;
    v.n_slots = n_slots;
    v.Db = Db;
    v.Da = Da;
    v.M = op->M;
    v.identity = ident;
    v.dt = x->dt;
    v.slot.assign(2 * t->n, nullptr);
    for (int u = 0; u < t->n; ++u) {
      if (u == t->root) continue;
      const size_t bytes = (size_t)n_slots * v.Db[u] * (ident ? 1 : v.M[u]) * v.Da[u] * es;
      for (int d = 0; d < (down ? 2 : 1); ++d)
        if (!alloc(e, &v.slot[2 * u + d], bytes)) return false;
    }
    return true;
  };
  std::vector<int> ones_b(t->n, 1);
  std::vector<int32_t> hl(kn), hj(kn), hz(std::max(k, kn), 0), hi(k);
  for (int p = 0; p < kn; ++p) {
    hl[p] = p % n_sketch;
    hj[p] = p / n_sketch;
  }
  for (int j = 0; j < k; ++j) hi[j] = j;
  std::vector<double> ones_d(n_sketch, 1.0);
  std::vector<float> ones_f(n_sketch, 1.0f);
  const size_t xs_b = (size_t)k * e->max_d * e->max_rest * es, ss_b = (size_t)kn * e->max_rest * es,
               aw_b = (size_t)k * (e->max_d + n_sketch) * e->max_rest * es;
  if (!make(e->senv, kn, ones_b, x->D, false, true) || !make(e->hav, k, y->D, x->D, false, false) ||
      !make(e->bxv, k, y->D, x->D, true, false) || !make(e->idv, 1, x->D, x->D, true, false) ||
      !alloc(e, &e->ones, (size_t)n_sketch * es) || !alloc(e, &e->xs, xs_b) || !alloc(e, &e->ss, ss_b) ||
      !alloc(e, &e->aw, aw_b) || !alloc(e, (void**)&e->d_l, (size_t)kn * 4) ||
      !alloc(e, (void**)&e->d_j, (size_t)kn * 4) || !upload_sync(e->d_l, hl.data(), hl.size() * 4, ctx->stream) ||
      !alloc(e, (void**)&e->d_zero, hz.size() * 4) || !alloc(e, (void**)&e->d_iota, (size_t)k * 4) ||
      !upload_sync(e->d_j, hj.data(), hj.size() * 4, ctx->stream) ||
      !upload_sync(e->d_zero, hz.data(), hz.size() * 4, ctx->stream) ||
      !upload_sync(e->d_iota, hi.data(), hi.size() * 4, ctx->stream) ||
      !upload_sync(e->ones, es == 8 ? (const void*)ones_d.data() : (const void*)ones_f.data(), (size_t)n_sketch * es,
                   ctx->stream)) {
    delete e;
    return api_fail(ctx, TTN_E_DEVICE, "allocation failed");
  }
  // delta environments of the open parent legs
  const int ct = x->dt == TTN_F64 ? 0 : 1;
  for (int u = 0; u < t->n; ++u) {
    if (u == t->root) continue;
    if (launch_set_identity(ct, e->idv.slot[2 * u], x->D[u], 1, ctx->stream) != hipSuccess) {
      delete e;
      return api_fail(ctx, TTN_E_LAUNCH, "identity environment launch failed");
    }
  }
  *out = e;
  return TTN_OK;
}

ttn_status ttn_expand_destroy(ttn_expand* e) {
  if (e) (void)hipStreamSynchronize(e->ctx->stream);
  delete e;
  return TTN_OK;
}

ttn_status ttn_expand_apply(ttn_ctx* ctx, ttn_expand* e, const void* const* omega) {
  if (!ctx || !e || !omega || e->ctx != ctx) return api_fail(ctx, TTN_E_ARG, "bad arguments");
  const ttn_tree* t = e->t;
  const int k = e->k, n = e->n, kn = k * n;
  const int ct = e->x->dt == TTN_F64 ? 0 : 1;
  for (int u = 0; u < t->n; ++u) {
    if (t->phys[u] > 1 && !omega[u]) return api_fail(ctx, TTN_E_ARG, "missing test matrix at a physical node");
    e->om.ptr[u] = t->phys[u] > 1 ? const_cast<void*>(omega[u]) : e->ones;
  }
  ttn_status r = TTN_OK;
  // 1. sketch environments <omega_l|H|x_j> (items p = j n + l)
  for (int u : e->post)
    if (u != t->root) {
      r = ttno_env_update(ctx, t, e->op, &e->om, e->x, kn, e->d_l, e->d_j, u, t->parent[u], &e->senv, e->compute);
      if (r != TTN_OK) return r;
    }
  for (auto it = e->post.rbegin(); it != e->post.rend(); ++it)
    for (int c : t->ch[*it]) {
      r = ttno_env_update(ctx, t, e->op, &e->om, e->x, kn, e->d_l, e->d_j, *it, c, &e->senv, e->compute);
      if (r != TTN_OK) return r;
    }
  // 2. leaves to root
  for (int u : e->post) {
    const int p = t->parent[u];
    if (p < 0) {
      // 3. the root: x_root in the children's new bases
      r = heff_apply_block(ctx, t, nullptr, &e->bxv, u, k, nullptr, nullptr, nullptr, nullptr, e->x->ptr[u], k,
                           e->y->ptr[u], TTN_HEFF_NO_SHIFT, e->compute);
      if (r != TTN_OK) return r;
      continue;
    }
    const int Du = e->x->D[u], Dn = e->y->D[u];
    int64_t rest = t->phys[u];
    for (int c : t->ch[u]) rest *= e->y->D[c];
    // a. X_u = x_u with the children legs through <y|x>, the parent leg open
    {
      ttn_envs mix;
      mix.t = t;
      mix.n_slots = k;
      mix.Db = e->y->D;
      mix.Db[u] = Du;
      mix.Da = e->x->D;
      mix.M = e->op->M;
      mix.identity = true;
      mix.dt = e->x->dt;
      mix.slot.assign(2 * t->n, nullptr);
      ctx->leg_tabs.clear();
      for (int c : t->nb[u]) {
        if (c == p) {
          mix.slot[ttn_envs::dslot(t, p, u)] = e->idv.slot[2 * u];
          ctx->leg_tabs.push_back({e->d_zero, 1});
        } else {
          mix.slot[ttn_envs::dslot(t, c, u)] = e->bxv.slot[ttn_envs::dslot(t, c, u)];
          ctx->leg_tabs.push_back({nullptr, k});
        }
      }
      r = ttn::heff_apply_rows(ctx, t, nullptr, &mix, u, k, nullptr, nullptr, nullptr, k, nullptr, nullptr,
                               e->x->ptr[u], k, e->xs, TTN_HEFF_NO_SHIFT, e->compute);
      ctx->leg_tabs.clear();
      if (r != TTN_OK) return r;
    }
    // its QR, Q left in place
    {
      std::vector<int> dims{Du};
      for (int c : t->ch[u]) dims.push_back(e->y->D[c]);
      dims.push_back(t->phys[u]);
      int64_t cs = 0;
      int m = 0;
      ttn_status code = TTN_OK;
      const int32_t* ro = leg_rows_table(ctx, dims, 0, cs, m, code);
      if (!ro) return code;
      const size_t work = (size_t)k * 2 * m * Du * sizeof(double);
      const size_t rbytes = (size_t)k * (Du * Du + Du) * sizeof(double);
      auto al = [](size_t v) { return (v + 255) / 256 * 256; };
      if (al(work) + al(rbytes) > ctx->ws_bytes) return api_fail(ctx, TTN_E_WORKSPACE, "workspace too small for QR");
      ctx->ws_last_plan = nullptr;
      double* wk = (double*)ctx->ws;
      double* R = (double*)((char*)ctx->ws + al(work));
      hipError_t he = launch_qr(ct, e->xs, (int64_t)Du * rest, ro, m, Du, cs, wk, R, k, ctx->d_flag, ctx->stream);
      if (he != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(he));
    }
    // b. the local sketch of H x: children legs through <y|H|x> (slot j), the
    //    parent leg through the sketch environment parent -> u (slot j n + l)
    {
      ttn_envs mix;
      mix.t = t;
      mix.n_slots = kn;
      mix.Db = e->y->D;
      mix.Db[u] = 1;
      mix.Da = e->x->D;
      mix.M = e->op->M;
      mix.dt = e->x->dt;
      mix.slot.assign(2 * t->n, nullptr);
      mix.slot[ttn_envs::dslot(t, p, u)] = e->senv.slot[ttn_envs::dslot(t, p, u)];
      ctx->leg_tabs.clear();
      for (int c : t->nb[u]) {
        if (c == p) {
          ctx->leg_tabs.push_back({nullptr, kn});
        } else {
          mix.slot[ttn_envs::dslot(t, c, u)] = e->hav.slot[ttn_envs::dslot(t, c, u)];
          ctx->leg_tabs.push_back({e->d_j, k});
        }
      }
      r = ttn::heff_apply_rows(ctx, t, e->op, &mix, u, kn, nullptr, e->d_j, nullptr, kn, nullptr, nullptr,
                               e->x->ptr[u], k, e->ss, TTN_HEFF_NO_SHIFT, e->compute);
      ctx->leg_tabs.clear();
      if (r != TTN_OK) return r;
    }
    // c.-d. the rank-revealing completion into y_u
    {
      hipError_t he = launch_expand_complete(ct, e->xs, (int64_t)Du * rest, e->ss, (int64_t)n * rest, e->aw,
                                             (int64_t)(Du + n) * rest, e->y->ptr[u], (int64_t)Dn * rest, Du, n,
                                             Dn - Du, (int)rest, k, ctx->stream);
      if (he != hipSuccess) return api_fail(ctx, TTN_E_LAUNCH, hipGetErrorString(he));
    }
    // e. <y|x> and <y|H|x> across the edge u -> parent
    r = ttno_env_update(ctx, t, nullptr, e->y, e->x, k, e->d_iota, e->d_iota, u, p, &e->bxv, e->compute);
    if (r != TTN_OK) return r;
    r = ttno_env_update(ctx, t, e->op, e->y, e->x, k, e->d_iota, e->d_iota, u, p, &e->hav, e->compute);
    if (r != TTN_OK) return r;
  }
  return TTN_OK;
}

}  // extern "C"
