// C ABI: handles, validation and the contraction entry points
// (ttno_env_update, ttno_env_close, heff_apply_block).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <new>
#include <sstream>

#include "internal.h"

using namespace ttn;

namespace ttn {

namespace {
std::atomic<int64_t> g_allocs{0};  // device and pinned-host allocations made by the library
constexpr size_t kPoolEntries = (size_t)16 << 20;  // 64 MiB of int32 table entries per context
}  // namespace

bool dev_malloc(void** p, size_t bytes) {
  if (hipMalloc(p, bytes ? bytes : 16) != hipSuccess) return false;
  g_allocs.fetch_add(1);
  return true;
}

bool pinned_malloc(void** p, size_t bytes) {
  if (hipHostMalloc(p, bytes ? bytes : 16, hipHostMallocDefault) != hipSuccess) return false;
  g_allocs.fetch_add(1);
  return true;
}

const int32_t* pool_upload(ttn_ctx* ctx, std::vector<int32_t>&& h, ttn_status& code) {
  const size_t n = h.empty() ? 1 : h.size();
  const size_t start = (ctx->pool_used + 63) / 64 * 64;  // 256-byte alignment
  if (start + n > ctx->pool_cap) {
    code = api_fail(ctx, TTN_E_WORKSPACE, "offset-table pool exhausted (64 MiB per context)");
    return nullptr;
  }
  if (h.empty()) h.push_back(0);
  ctx->pool_host.push_back(std::move(h));
  const std::vector<int32_t>& keep = ctx->pool_host.back();
  int32_t* d = ctx->pool + start;
  if (hipMemcpyAsync(d, keep.data(), keep.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream) !=
      hipSuccess) {
    code = api_fail(ctx, TTN_E_DEVICE, "offset-table upload failed");
    return nullptr;
  }
  ctx->pool_used = start + n;
  return d;
}

bool prof_selected(const ttn_ctx* ctx, const std::string& key) {
  if (ctx->prof_filter.empty()) return true;
  for (const std::string& f : ctx->prof_filter)
    if (key.compare(0, f.size(), f) == 0) return true;
  return false;
}

}  // namespace ttn

namespace {

thread_local std::string g_err;  // for calls without a context

ttn_status fail(ttn_ctx* ctx, ttn_status code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  g_err = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                                  \
  do {                                                                                     \
    hipError_t _e = (call);                                                                \
    if (_e != hipSuccess) return fail(ctx, TTN_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(_e)); \
  } while (0)

// engine compute types: 0 f64, 1 f32, 2 f32 storage with bf16 MFMA, 3 f64 storage with f32 MFMA
int ctype_of(ttn_dtype compute) {
  return compute == TTN_F64 ? 0 : (compute == TTN_F32 ? 1 : (compute == TTN_BF16 ? 2 : 3));
}
size_t esize(int ct) { return (ct == 0 || ct == 3) ? 8 : 4; }
// element type of the storage for the non-GEMM kernels (0 double, 1 float)
int stype(int ct) { return (ct == 0 || ct == 3) ? 0 : 1; }

bool dtype_ok(ttn_dtype storage, ttn_dtype compute) {
  if (compute == TTN_F64 || compute == TTN_F64_F32) return storage == TTN_F64;
  return storage == TTN_F32;
}

// row-major strides of dims, dropping size-1 legs: returns (labels, strides)
void add_tensor(std::vector<Tensor>& v, const std::vector<int>& labs, const std::vector<int>& dms, int batched,
                std::map<int, int>& dims) {
  Tensor t;
  int64_t s = 1;
  std::vector<int64_t> st(labs.size());
  for (int i = (int)labs.size() - 1; i >= 0; --i) {
    st[i] = s;
    s *= dms[i];
  }
  for (size_t i = 0; i < labs.size(); ++i) {
    auto it = dims.find(labs[i]);
    if (it == dims.end()) dims[labs[i]] = dms[i];
    if (dms[i] == 1) continue;
    t.lab.push_back(labs[i]);
    t.str.push_back(st[i]);
  }
  t.batched = batched;
  v.push_back(t);
}

void out_layout(const std::vector<int>& labs, const std::vector<int>& dms, std::vector<int>& ol,
                std::vector<int64_t>& os) {
  int64_t s = 1;
  std::vector<int64_t> st(labs.size());
  for (int i = (int)labs.size() - 1; i >= 0; --i) {
    st[i] = s;
    s *= dms[i];
  }
  ol.clear();
  os.clear();
  for (size_t i = 0; i < labs.size(); ++i) {
    if (dms[i] == 1) continue;
    ol.push_back(labs[i]);
    os.push_back(st[i]);
  }
}

// Execute a plan over batch items [0, nb): inputs[i] addressing, final output
// addressing and epilogue.  Chunks the batch to the workspace.
// Autotuner: run one stage with every tile shape (the stage overwrites its
// output, so repeats are harmless), time each with events, keep the fastest.
ttn_status tune_stage(ttn_ctx* ctx, Plan& P, size_t s, int ct, const OpAddr& A, const OpAddr& B, const OpAddr& C,
                      const Epilogue& e, int z0, int cnt) {
  Step& st = P.steps[s];
  std::vector<int> cand{0, 1, 2, 3, 4, 5, 6};
  if (splitk_eligible(st.g, ct)) cand.push_back(8);
  if (narrow_eligible(st.g, ct)) cand.push_back(9);
  if (tn_eligible(st.g, ct))
    for (int c = 10; c <= 16; ++c) cand.push_back(c);
  hipEvent_t ev[2];
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
    return fail(ctx, TTN_E_DEVICE, "hipEventCreate failed");
  const int orig = st.g.tile;
  int best = orig;
  float best_ms = 1e30f;
  std::ostringstream log;
  log << P.key << "|" << s << "|" << st.g.M << "|" << st.g.N << "|" << st.g.K << "|" << cnt;
  std::ostringstream times;
  for (int c : cand) {
    st.g.tile = c;
    float ms = 0;
    for (int rep = 0; rep < 2; ++rep) {  // the first launch warms caches and code
      (void)hipEventRecord(ev[0], ctx->stream);
      hipError_t he = launch_gemm(ct, st.g, A, B, C, e, z0, cnt, ctx->d_flag, ctx->stream);
      (void)hipEventRecord(ev[1], ctx->stream);
      if (he != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        return fail(ctx, TTN_E_LAUNCH, "autotune launch failed");
      }
      (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    }
    times << "|" << c << ":" << (int)(ms * 1000.0f);
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  st.g.tile = best;
  st.tuned = true;
  log << "|" << orig << "->" << best << times.str() << "\n";
  ctx->tune_log += log.str();
  return TTN_OK;
}

ttn_status exec_plan(ttn_ctx* ctx, Plan& P, int ct, const std::vector<OpAddr>& inputs, const OpAddr& out,
                     const Epilogue& ep, int nb, const std::vector<int64_t>& in_elems, int64_t out_elems,
                     size_t ws_off_bytes = 0) {
  const size_t es = esize(ct);
  {
    std::string why;
    if (!check_plan_bounds(P, in_elems, out_elems, why)) return fail(ctx, TTN_E_SHAPE, why);
  }
  const size_t avail = ctx->ws_bytes > ws_off_bytes ? (ctx->ws_bytes - ws_off_bytes) / es : 0;
  if ((size_t)P.ws_shared > avail) return fail(ctx, TTN_E_WORKSPACE, "workspace too small for shared intermediates");
  int64_t chunk = nb;
  if (P.ws_per_item > 0) {
    chunk = (int64_t)((avail - P.ws_shared) / P.ws_per_item);
    if (chunk < 1) return fail(ctx, TTN_E_WORKSPACE, "workspace too small for one batch item");
    chunk = std::min<int64_t>(chunk, nb);
  }
  char* ws = (char*)ctx->ws + ws_off_bytes;
  // stages whose operands do not depend on input 0 (X of an H_eff product)
  std::vector<char> dep_x((size_t)P.n_in + P.steps.size(), 0);
  dep_x[0] = 1;
  {
    int nid = P.n_in;
    for (const Step& st : P.steps)
      if (st.out >= 0) dep_x[nid++] = dep_x[st.a] || (st.b >= 0 && dep_x[st.b]);
  }
  auto step_dep_x = [&](const Step& st) { return dep_x[st.a] || (st.b >= 0 && dep_x[st.b]); };
  std::vector<const void*> in_bases;
  for (const OpAddr& o : inputs) in_bases.push_back(o.base);
  in_bases.push_back(out.base);
  // every X-independent intermediate of this plan is still in the workspace
  // (same plan, same inputs, same single chunk, nothing else ran since)
  const bool reuse = ctx->reuse_free && chunk >= nb && ctx->ws_last_plan == (const void*)&P &&
                     ctx->ws_last_nb == nb && ctx->ws_last_base == (const void*)ws &&
                     ctx->ws_last_inputs.size() == in_bases.size() &&
                     std::equal(in_bases.begin() + 1, in_bases.end() - 1, ctx->ws_last_inputs.begin() + 1);
  ctx->ws_last_plan = nullptr;  // the workspace is about to change
  double skipped = 0;
  if (reuse)
    for (const Step& st : P.steps)
      if (st.out >= 0 && !step_dep_x(st)) skipped += st.batched ? st.flops * nb : st.flops;
  ctx->flops_done += P.flops_per_item * nb + P.flops_shared - skipped;
  // shared intermediates are computed once (first chunk) and kept
  bool shared_done = false;
  for (int z0 = 0; z0 < nb; z0 += (int)chunk) {
    const int nz = (int)std::min<int64_t>(chunk, nb - z0);
    // addresses of intermediates for this chunk
    std::vector<OpAddr> inter;
    int shared_i = 0;
    (void)shared_i;
    size_t ib = 0;
    for (size_t s = 0; s < P.steps.size(); ++s) {
      const Step& st = P.steps[s];
      if (st.out < 0) continue;
      OpAddr o;
      const int64_t padded = (st.out_size + 63) / 64 * 64;
      if (st.batched) {
        o.base = ws + ((size_t)P.ws_shared + (size_t)P.inter_off[ib] * nz) * es;
        o.bstride = padded;
        o.local = true;
      } else {
        o.base = ws + (size_t)P.inter_off[ib] * es;
        o.shared = true;
      }
      inter.push_back(o);
      ++ib;
    }
    auto addr = [&](int id) -> OpAddr {
      if (id < P.n_in) return inputs[id];
      return inter[id - P.n_in];
    };
    for (size_t s = 0; s < P.steps.size(); ++s) {
      const Step& st = P.steps[s];
      if (!st.batched && shared_done) continue;
      if (reuse && st.out >= 0 && !step_dep_x(st)) continue;  // still in the workspace
      if (st.kind == 1) {  // relayout of a shared input into its slot
        hipError_t he = launch_relayout(ct, addr(st.a).base, st.g.a_om, st.g.a_ok, st.g.M, st.g.K,
                                        (void*)addr(st.out).base, ctx->stream, ctx->gate);
        if (he != hipSuccess) return fail(ctx, TTN_E_LAUNCH, std::string("relayout launch: ") + hipGetErrorString(he));
        continue;
      }
      const OpAddr A = addr(st.a), B = addr(st.b);
      const bool last = st.out < 0;
      OpAddr C = last ? out : addr(st.out);
      Epilogue e = last ? ep : Epilogue();
      const int cnt = st.batched ? nz : 1;
      if (ctx->autotune && !st.tuned && !e.accum && !ctx->profile) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(ctx->stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
          ttn_status tr = tune_stage(ctx, P, s, ct, A, B, C, e, st.batched ? z0 : 0, cnt);
          if (tr != TTN_OK) return tr;
        }
      }
      ttn_prof_rec* rec = nullptr;
      if (ctx->profile && ctx->prof.size() < 200000 && prof_selected(ctx, P.key)) {
        ctx->prof.emplace_back();
        rec = &ctx->prof.back();
        rec->key = P.key;
        rec->step = (int)s;
        rec->kernel = gemm_kernel_name(ct, st.g);
        rec->flops = st.flops * cnt;
        {
          const double mk = (double)st.g.M * st.g.K, kn = (double)st.g.K * st.g.N, mn = (double)st.g.M * st.g.N;
          const double per = (A.shared ? 0.0 : mk) + (B.shared ? 0.0 : kn) +
                             mn * (1.0 + (e.accum ? 1.0 : 0.0) + (e.D.base ? 1.0 : 0.0));
          rec->bytes = (double)es * (per * cnt + (A.shared ? mk : 0.0) + (B.shared ? kn : 0.0));
        }
        rec->M = st.g.M;
        rec->N = st.g.N;
        rec->K = st.g.K;
        rec->nz = cnt;
        if (hipEventCreate(&rec->a) != hipSuccess || hipEventCreate(&rec->b) != hipSuccess)
          return fail(ctx, TTN_E_DEVICE, "hipEventCreate failed");
        (void)hipEventRecord(rec->a, ctx->stream);
      }
      hipError_t he = launch_gemm(ct, st.g, A, B, C, e, st.batched ? z0 : 0, cnt, ctx->d_flag, ctx->stream, ctx->gate);
      if (he != hipSuccess) return fail(ctx, TTN_E_LAUNCH, std::string("gemm launch: ") + hipGetErrorString(he));
      if (rec) (void)hipEventRecord(rec->b, ctx->stream);
    }
    shared_done = true;
  }
  if (chunk >= nb) {
    ctx->ws_last_plan = (const void*)&P;
    ctx->ws_last_nb = nb;
    ctx->ws_last_base = (const void*)ws;
    ctx->ws_last_inputs = in_bases;
  }
  return TTN_OK;
}

int64_t w_elems(const ttn_tree* t, const ttn_ttno* op, int u) {
  int64_t n = (int64_t)t->phys[u] * t->phys[u];
  for (int c : t->nb[u]) n *= op->bond(u, c);
  return n;
}

// ---- network builders (labels: leg i -> b 3i, w 3i+1, a 3i+2; p 3k, q 3k+1)

struct Net {
  std::vector<Tensor> in;
  std::map<int, int> dims;
  std::vector<int> out_lab;
  std::vector<int64_t> out_str;
  std::string key;
};

// heff at node u: inputs [X, (W), E_0..E_{k-1}], output Y[b..., p]
bool build_heff_net(const ttn_tree* t, const ttn_ttno* op, const ttn_envs* env, int u, Net& net, std::string& why) {
  const int kap = (int)t->nb[u].size();
  const int d = t->phys[u];
  const int P = 3 * kap, Q = op ? 3 * kap + 1 : 3 * kap;
  std::vector<int> xl, xd, wl, wd, yl, yd;
  std::ostringstream key;
  key << "heff:" << u << ":" << (op ? 1 : 0);
  for (int i = 0; i < kap; ++i) {
    const int c = t->nb[u][i];
    xl.push_back(3 * i + 2);
    xd.push_back(env->ea(c, u));
    yl.push_back(3 * i);
    yd.push_back(env->eb(c, u));
    if (op) {
      wl.push_back(3 * i + 1);
      wd.push_back(op->bond(u, c));
      if (env->em(c, u) != op->bond(u, c)) {
        why = "environment operator bond differs from the TTNO bond";
        return false;
      }
    } else if (env->em(c, u) != 1) {
      why = "identity operator needs environments with operator bond 1";
      return false;
    }
  }
  xl.push_back(Q);
  xd.push_back(d);
  yl.push_back(P);
  yd.push_back(d);
  add_tensor(net.in, xl, xd, 1, net.dims);
  if (op) {
    wl.push_back(P);
    wd.push_back(d);
    wl.push_back(Q);
    wd.push_back(d);
    add_tensor(net.in, wl, wd, 0, net.dims);
  }
  for (int i = 0; i < kap; ++i) {
    const int c = t->nb[u][i];
    std::vector<int> el{3 * i, 3 * i + 1, 3 * i + 2};
    std::vector<int> ed{env->eb(c, u), env->em(c, u), env->ea(c, u)};
    add_tensor(net.in, el, ed, 1, net.dims);
    key << ":" << ed[0] << "x" << ed[1] << "x" << ed[2];
  }
  key << ":d" << d;
  out_layout(yl, yd, net.out_lab, net.out_str);
  net.key = key.str();
  return true;
}

// env update u -> v: inputs [bra, (W), ket, E_i (i != iv)], output E[b_iv, w_iv, a_iv]
bool build_env_net(const ttn_tree* t, const ttn_ttno* op, const ttn_block* bra, const ttn_block* ket,
                   const ttn_envs* env, int u, int v, Net& net, std::string& why) {
  const int kap = (int)t->nb[u].size();
  const int d = t->phys[u];
  const int iv = t->leg_of(u, v);
  const int P = 3 * kap, Q = op ? 3 * kap + 1 : 3 * kap;
  std::ostringstream key;
  key << "env:" << u << ">" << v << ":" << (op ? 1 : 0);
  std::vector<int> bl, bd, kl, kd, wl, wd;
  for (int i = 0; i < kap; ++i) {
    const int c = t->nb[u][i];
    bl.push_back(3 * i);
    bd.push_back(bra->bond(u, c));
    kl.push_back(3 * i + 2);
    kd.push_back(ket->bond(u, c));
    if (op) {
      wl.push_back(3 * i + 1);
      wd.push_back(op->bond(u, c));
    }
    if (env->eb(u, c) != bra->bond(u, c) || env->ea(u, c) != ket->bond(u, c)) {
      why = "environment bonds differ from the bra/ket bonds";
      return false;
    }
    if (env->em(u, c) != (op ? op->bond(u, c) : 1)) {
      why = "environment operator bond differs from the operator";
      return false;
    }
  }
  bl.push_back(P);
  bd.push_back(d);
  kl.push_back(Q);
  kd.push_back(d);
  add_tensor(net.in, bl, bd, 1, net.dims);
  if (op) {
    wl.push_back(P);
    wd.push_back(d);
    wl.push_back(Q);
    wd.push_back(d);
    add_tensor(net.in, wl, wd, 0, net.dims);
  }
  add_tensor(net.in, kl, kd, 1, net.dims);
  for (int i = 0; i < kap; ++i) {
    if (i == iv) continue;
    const int c = t->nb[u][i];
    std::vector<int> el{3 * i, 3 * i + 1, 3 * i + 2};
    std::vector<int> ed{env->eb(c, u), env->em(c, u), env->ea(c, u)};
    add_tensor(net.in, el, ed, 1, net.dims);
    key << ":" << ed[0] << "x" << ed[1] << "x" << ed[2];
  }
  key << ":" << bra->bond(u, v) << "," << env->em(u, v) << "," << ket->bond(u, v) << ":d" << d;
  std::vector<int> ol{3 * iv, 3 * iv + 1, 3 * iv + 2};
  std::vector<int> od{env->eb(u, v), env->em(u, v), env->ea(u, v)};
  out_layout(ol, od, net.out_lab, net.out_str);
  net.key = key.str();
  return true;
}

// The plan cache key ends with the whole network written out (every operand's
// labels, extents, strides and batching, the output's labels and strides; no
// '|', which separates the fields of the profile and autotune reports):
// the readable prefix alone does not say through which leg an environment
// leaves, and contexts serve several trees whose node numbers coincide.
void net_signature(const Net& net, std::ostringstream& k) {
  for (const Tensor& t : net.in) {
    k << ";" << t.batched;
    for (size_t i = 0; i < t.lab.size(); ++i) k << "," << t.lab[i] << "=" << net.dims.at(t.lab[i]) << "/" << t.str[i];
  }
  k << ";>";
  for (size_t i = 0; i < net.out_lab.size(); ++i)
    k << "," << net.out_lab[i] << "=" << net.dims.at(net.out_lab[i]) << "/" << net.out_str[i];
}

Plan* get_plan(ttn_ctx* ctx, const Net& net, int ct, double batch, ttn_status& code) {
  std::ostringstream k;
  k << net.key << ":ct" << ct << ":b" << (batch <= 1 ? 0 : (batch < 256 ? 1 : 2)) << "#";
  net_signature(net, k);
  auto it = ctx->plans.find(k.str());
  if (it != ctx->plans.end()) return it->second.get();
  Status st;
  auto p = make_plan(net.in, net.dims, net.out_lab, net.out_str, batch, ct, st);
  if (!p) {
    code = fail(ctx, st.code, st.msg);
    return nullptr;
  }
  const int32_t* d_tabs = pool_upload(ctx, std::move(p->h_tabs), code);
  if (!d_tabs) return nullptr;
  bind_plan_tables(*p, d_tabs);
  Plan* raw = p.get();
  raw->key = k.str();
  ctx->plans[k.str()] = std::move(p);
  return raw;
}

}  // namespace

namespace ttn {
ttn_status api_fail(ttn_ctx* ctx, ttn_status code, const std::string& msg) { return fail(ctx, code, msg); }
}  // namespace ttn

// ================================================================== housekeeping

extern "C" {

const char* ttn_version(void) { return "ttn-mi355x 0.1 (gfx950)"; }

const char* ttn_last_error(const ttn_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

ttn_status ttn_ctx_create(int device, void* hip_stream, size_t workspace_bytes, ttn_ctx** out) {
  if (!out) return fail(nullptr, TTN_E_ARG, "out is null");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
    return fail(nullptr, TTN_E_DEVICE, "no such HIP device");
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, TTN_E_DEVICE, "hipSetDevice failed");
  ttn_ctx* c = new (std::nothrow) ttn_ctx();
  if (!c) return fail(nullptr, TTN_E_ARG, "out of host memory");
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->ws_bytes = workspace_bytes ? workspace_bytes : ((size_t)1 << 30);
  if (!dev_malloc(&c->ws, c->ws_bytes)) {
    delete c;
    return fail(nullptr, TTN_E_DEVICE, "workspace hipMalloc failed");
  }
  if (!dev_malloc((void**)&c->pool, kPoolEntries * sizeof(int32_t))) {
    (void)hipFree(c->ws);
    delete c;
    return fail(nullptr, TTN_E_DEVICE, "table pool hipMalloc failed");
  }
  c->pool_cap = kPoolEntries;
  if (!dev_malloc((void**)&c->d_flag, 4 * sizeof(int)) ||
      hipMemsetAsync(c->d_flag, 0, 4 * sizeof(int), c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipFree(c->ws);
    (void)hipFree(c->pool);
    delete c;
    return fail(nullptr, TTN_E_DEVICE, "flag hipMalloc failed");
  }
  if (!noalloc_scratch_setup(device, &c->scratch)) c->scratch = nullptr;  // heff_apply_block_noalloc reports it
  *out = c;
  return TTN_OK;
}

ttn_status ttn_ctx_set_stream(ttn_ctx* ctx, void* s) {
  if (!ctx) return fail(nullptr, TTN_E_ARG, "null context");
  // table uploads already enqueued are ordered on the old stream only
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->stream = (hipStream_t)s;
  return TTN_OK;
}

ttn_status ttn_alloc_count(int64_t* out) {
  if (!out) return fail(nullptr, TTN_E_ARG, "null argument");
  *out = g_allocs.load();
  return TTN_OK;
}

ttn_status ttn_ctx_sync(ttn_ctx* ctx) {
  if (!ctx) return fail(nullptr, TTN_E_ARG, "null context");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  int f[4];
  HIPCHK(ctx, hipMemcpyAsync(f, ctx->d_flag, sizeof(f), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (f[0] || f[1] || f[2] || f[3]) {
    HIPCHK(ctx, hipMemsetAsync(ctx->d_flag, 0, sizeof(f), ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (f[2]) return fail(ctx, TTN_E_ARG, "a pair / row index table held an out-of-range index (clamped)");
    if (f[0]) return fail(ctx, TTN_E_NONFINITE, "a kernel produced a non-finite value");
    if (f[3]) return fail(ctx, TTN_E_NOCONV, "the symmetric eigensolver of Rayleigh-Ritz did not converge");
    return fail(ctx, TTN_E_NOT_PD, "overlap matrix not positive definite (SVQB disabled)");
  }
  return TTN_OK;
}

ttn_status ttn_ctx_destroy(ttn_ctx* ctx) {
  if (!ctx) return TTN_OK;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& c : ctx->calls) {
    (void)hipEventDestroy(c.a);
    (void)hipEventDestroy(c.b);
  }
  for (auto& r : ctx->prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  ctx->plans.clear();
  ctx->tables.clear();
  if (ctx->pool) (void)hipFree(ctx->pool);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->d_flag) (void)hipFree(ctx->d_flag);
  delete ctx;
  return TTN_OK;
}

ttn_status ttn_tree_create(int32_t n, const int32_t* parent, const int32_t* phys, ttn_tree** out) {
  if (!out || !parent || !phys || n <= 0) return fail(nullptr, TTN_E_ARG, "bad tree arguments");
  ttn_tree* t = new (std::nothrow) ttn_tree();
  if (!t) return fail(nullptr, TTN_E_ARG, "out of host memory");
  t->n = n;
  t->parent.assign(parent, parent + n);
  t->phys.assign(phys, phys + n);
  t->ch.assign(n, {});
  int roots = 0;
  for (int u = 0; u < n; ++u) {
    if (phys[u] < 1) {
      delete t;
      return fail(nullptr, TTN_E_ARG, "physical dimension must be >= 1");
    }
    if (parent[u] < 0) {
      t->root = u;
      ++roots;
    } else if (parent[u] >= n || parent[u] == u) {
      delete t;
      return fail(nullptr, TTN_E_ARG, "parent index out of range");
    } else {
      t->ch[parent[u]].push_back(u);
    }
  }
  if (roots != 1) {
    delete t;
    return fail(nullptr, TTN_E_ARG, "tree needs exactly one root");
  }
  // acyclic: every node reaches the root
  for (int u = 0; u < n; ++u) {
    int x = u, steps = 0;
    while (parent[x] >= 0 && steps <= n) {
      x = parent[x];
      ++steps;
    }
    if (steps > n) {
      delete t;
      return fail(nullptr, TTN_E_ARG, "parent array has a cycle");
    }
  }
  t->nb.assign(n, {});
  for (int u = 0; u < n; ++u) {
    if (parent[u] >= 0) t->nb[u].push_back(parent[u]);
    for (int c : t->ch[u]) t->nb[u].push_back(c);
    if (t->nb[u].size() > 4) {
      delete t;
      return fail(nullptr, TTN_E_ARG, "nodes with more than 4 neighbours are not supported");
    }
  }
  *out = t;
  return TTN_OK;
}

ttn_status ttn_tree_destroy(ttn_tree* t) {
  delete t;
  return TTN_OK;
}

ttn_status ttn_ttno_create(ttn_ctx* ctx, const ttn_tree* t, const int32_t* op_bond, ttn_dtype dtype, void* const* W,
                           ttn_ttno** out) {
  if (!ctx || !t || !op_bond || !W || !out) return fail(ctx, TTN_E_ARG, "null argument");
  if (dtype != TTN_F64 && dtype != TTN_F32) return fail(ctx, TTN_E_DTYPE, "TTNO storage must be F64 or F32");
  ttn_ttno* o = new (std::nothrow) ttn_ttno();
  o->t = t;
  o->M.assign(op_bond, op_bond + t->n);
  o->dt = dtype;
  o->W.assign(W, W + t->n);
  for (int u = 0; u < t->n; ++u) {
    if (!o->W[u] || (u != t->root && o->M[u] < 1)) {
      delete o;
      return fail(ctx, TTN_E_ARG, "missing TTNO tensor or bond");
    }
  }
  *out = o;
  return TTN_OK;
}

ttn_status ttn_ttno_destroy(ttn_ttno* o) {
  delete o;
  return TTN_OK;
}

ttn_status ttn_block_create(ttn_ctx* ctx, const ttn_tree* t, int32_t k, const int32_t* bond, ttn_dtype dtype,
                            void* const* node_ptr, ttn_block** out) {
  if (!ctx || !t || !bond || !node_ptr || !out || k < 1) return fail(ctx, TTN_E_ARG, "bad block arguments");
  if (dtype != TTN_F64 && dtype != TTN_F32) return fail(ctx, TTN_E_DTYPE, "block storage must be F64 or F32");
  ttn_block* b = new (std::nothrow) ttn_block();
  b->t = t;
  b->k = k;
  b->D.assign(bond, bond + t->n);
  b->dt = dtype;
  b->ptr.assign(node_ptr, node_ptr + t->n);
  b->size.resize(t->n);
  for (int u = 0; u < t->n; ++u) {
    if (u != t->root && b->D[u] < 1) {
      delete b;
      return fail(ctx, TTN_E_SHAPE, "bond dimension must be >= 1");
    }
    int64_t s = 1;
    for (int x : b->legdims(u)) s *= x;
    if (s > INT32_MAX / 2) {
      delete b;
      return fail(ctx, TTN_E_SHAPE, "node tensor too large");
    }
    b->size[u] = s;
    if (!b->ptr[u]) {
      delete b;
      return fail(ctx, TTN_E_ARG, "missing node buffer");
    }
  }
  *out = b;
  return TTN_OK;
}

ttn_status ttn_block_destroy(ttn_block* b) {
  delete b;
  return TTN_OK;
}

ttn_status ttn_block_node_size(const ttn_block* b, int32_t u, int64_t* s) {
  if (!b || !s || u < 0 || u >= b->t->n) return fail(nullptr, TTN_E_ARG, "bad node");
  *s = b->size[u];
  return TTN_OK;
}

ttn_status ttn_envs_create(ttn_ctx* ctx, const ttn_tree* t, int32_t n_slots, const int32_t* bra_bond,
                           const int32_t* op_bond, const int32_t* ket_bond, ttn_dtype dtype, void* const* slot_ptr,
                           ttn_envs** out) {
  if (!ctx || !t || n_slots < 1 || !bra_bond || !ket_bond || !slot_ptr || !out)
    return fail(ctx, TTN_E_ARG, "bad envs arguments");
  if (dtype != TTN_F64 && dtype != TTN_F32) return fail(ctx, TTN_E_DTYPE, "env storage must be F64 or F32");
  ttn_envs* e = new (std::nothrow) ttn_envs();
  e->t = t;
  e->n_slots = n_slots;
  e->Db.assign(bra_bond, bra_bond + t->n);
  e->Da.assign(ket_bond, ket_bond + t->n);
  e->identity = op_bond == nullptr;
  e->M = op_bond ? std::vector<int>(op_bond, op_bond + t->n) : std::vector<int>(t->n, 1);
  e->dt = dtype;
  e->slot.assign(slot_ptr, slot_ptr + 2 * t->n);
  *out = e;
  return TTN_OK;
}

ttn_status ttn_envs_destroy(ttn_envs* e) {
  delete e;
  return TTN_OK;
}

// ================================================================== hot path

ttn_status ttno_env_update(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_block* bra,
                           const ttn_block* ket, int32_t n_pairs, const int32_t* pair_bra, const int32_t* pair_ket,
                           int32_t node, int32_t toward, ttn_envs* envs, ttn_dtype compute) {
  if (!ctx || !t || !bra || !ket || !envs || !pair_bra || !pair_ket) return fail(ctx, TTN_E_ARG, "null argument");
  if (n_pairs < 0 || n_pairs > envs->n_slots) return fail(ctx, TTN_E_ARG, "n_pairs exceeds the env slots");
  if (node < 0 || node >= t->n || t->leg_of(node, toward) < 0) return fail(ctx, TTN_E_ARG, "toward is not a neighbour");
  if (bra->t != t || ket->t != t || envs->t != t || (op && op->t != t)) return fail(ctx, TTN_E_ARG, "tree mismatch");
  if (!dtype_ok(bra->dt, compute) || !dtype_ok(ket->dt, compute) || !dtype_ok(envs->dt, compute) ||
      (op && !dtype_ok(op->dt, compute)))
    return fail(ctx, TTN_E_DTYPE, "tensor dtype does not match the compute dtype");
  if ((op == nullptr) != envs->identity) return fail(ctx, TTN_E_ARG, "operator / environment kind mismatch");
  if (n_pairs == 0) return TTN_OK;
  const int u = node, v = toward;
  for (int c : t->nb[u])
    if (c != v && !envs->slot[ttn_envs::dslot(t, c, u)]) return fail(ctx, TTN_E_ARG, "missing incoming environment");
  if (!envs->slot[ttn_envs::dslot(t, u, v)]) return fail(ctx, TTN_E_ARG, "missing output environment");
  const int ct = ctype_of(compute);
  const int kap = (int)t->nb[u].size();
  {
    // three virtual legs, no physical leg, identity operator, FP32 storage,
    // equal bra / ket bonds <= 32: the fused kernel (intermediates in LDS)
    bool fuse = !op && kap == 3 && t->phys[u] == 1 && (ct == 1 || ct == 2) && bra->dt == TTN_F32 &&
                ket->dt == TTN_F32 && envs->dt == TTN_F32;
    const char* fe = getenv("TTN_FUSED_IENV");
    if (fe && fe[0] == '0') fuse = false;
    IEnv3Args fa;
    if (fuse) {
      for (int i = 0; i < 3 && fuse; ++i) {
        const int c = t->nb[u][i];
        fa.dim[i] = bra->bond(u, c);
        fuse = fa.dim[i] == ket->bond(u, c) && fa.dim[i] >= 1 && fa.dim[i] <= 32 && envs->eb(u, c) == fa.dim[i] &&
               envs->ea(u, c) == fa.dim[i];
      }
    }
    if (fuse) {
      const int iv = t->leg_of(u, v);
      fa.o = iv;
      fa.p = iv == 0 ? 1 : 0;
      fa.q = iv == 2 ? 1 : 2;
      fuse = ienv3_lds_bytes(fa.dim[fa.o], fa.dim[fa.p], fa.dim[fa.q]) <= IENV3_LDS_MAX;
    }
    if (fuse) {
      fa.stride[2] = 1;
      fa.stride[1] = fa.dim[2];
      fa.stride[0] = fa.dim[1] * fa.dim[2];
      fa.bra = (const float*)bra->ptr[u];
      fa.ket = (const float*)ket->ptr[u];
      fa.bra_size = bra->size[u];
      fa.ket_size = ket->size[u];
      fa.pb = pair_bra;
      fa.pk = pair_ket;
      fa.bra_rows = bra->k;
      fa.ket_rows = ket->k;
      const int cp = t->nb[u][fa.p], cq = t->nb[u][fa.q];
      fa.Ep = (const float*)envs->slot[ttn_envs::dslot(t, cp, u)];
      fa.Eq = (const float*)envs->slot[ttn_envs::dslot(t, cq, u)];
      fa.Eo = (float*)envs->slot[ttn_envs::dslot(t, u, v)];
      fa.ep_stride = envs->slot_elems(cp, u);
      fa.eq_stride = envs->slot_elems(cq, u);
      fa.eo_stride = envs->slot_elems(u, v);
      fa.n = n_pairs;
      fa.flag = ctx->d_flag;
      const double Do = fa.dim[fa.o], Dp = fa.dim[fa.p], Dq = fa.dim[fa.q];
      const double per = 2.0 * Do * Dp * Dq * (Dp + Dq + Do);  // the three products of the staged path
      ctx->flops_done += per * n_pairs;
      std::ostringstream key;
      key << "ienv:" << u << ">" << v;
      const std::string ks = key.str();
      // compulsory bytes: bra and ket tensors, two environments in, one out
      const double bytes = 4.0 * n_pairs * (2.0 * Do * Dp * Dq + Dp * Dp + Dq * Dq + Do * Do);
      ttn_prof_rec* pr = prof_begin(ctx, ks.c_str(), "ienv3_kernel", per * n_pairs, bytes, n_pairs);
      hipError_t he = launch_ienv3(fa, ctx->stream);
      prof_end(ctx, pr);
      if (he != hipSuccess) return fail(ctx, TTN_E_LAUNCH, std::string("fused environment: ") + hipGetErrorString(he));
      return TTN_OK;
    }
  }
  Net net;
  std::string why;
  if (!build_env_net(t, op, bra, ket, envs, u, v, net, why)) return fail(ctx, TTN_E_SHAPE, why);
  if (net.in.size() < 2) {
    // degenerate network (all legs trivial): not reachable for a tree node with a bond
    return fail(ctx, TTN_E_SHAPE, "degenerate environment network");
  }
  ttn_status code = TTN_OK;
  Plan* P = get_plan(ctx, net, ct, n_pairs, code);
  if (!P) return code;
  std::vector<OpAddr> in;
  std::vector<int64_t> ne;
  OpAddr a;
  a.base = bra->ptr[u];
  a.tab = pair_bra;
  a.tab_max = bra->k;
  a.bstride = bra->size[u];
  in.push_back(a);
  ne.push_back(bra->size[u]);
  if (op) {
    OpAddr w;
    w.base = op->W[u];
    w.shared = true;
    in.push_back(w);
    ne.push_back(w_elems(t, op, u));
  }
  OpAddr k;
  k.base = ket->ptr[u];
  k.tab = pair_ket;
  k.tab_max = ket->k;
  k.bstride = ket->size[u];
  in.push_back(k);
  ne.push_back(ket->size[u]);
  const int iv = t->leg_of(u, v);
  for (int i = 0; i < kap; ++i) {
    if (i == iv) continue;
    const int c = t->nb[u][i];
    OpAddr e;
    e.base = envs->slot[ttn_envs::dslot(t, c, u)];
    e.bstride = envs->slot_elems(c, u);
    in.push_back(e);
    ne.push_back(envs->slot_elems(c, u));
  }
  OpAddr o;
  o.base = envs->slot[ttn_envs::dslot(t, u, v)];
  o.bstride = envs->slot_elems(u, v);
  return exec_plan(ctx, *P, ct, in, o, Epilogue(), n_pairs, ne, envs->slot_elems(u, v));
}

ttn_status ttno_env_close(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_block* bra,
                          const ttn_block* ket, int32_t n_pairs, const int32_t* pair_bra, const int32_t* pair_ket,
                          int32_t node, const ttn_envs* envs, double* out, ttn_dtype compute) {
  if (!ctx || !t || !bra || !ket || !envs || !out || !pair_bra || !pair_ket) return fail(ctx, TTN_E_ARG, "null argument");
  if (node < 0 || node >= t->n) return fail(ctx, TTN_E_ARG, "bad node");
  if (n_pairs < 0 || n_pairs > envs->n_slots) return fail(ctx, TTN_E_ARG, "n_pairs exceeds the env slots");
  if (n_pairs == 0) return TTN_OK;
  if (t->nb[node].empty()) return fail(ctx, TTN_E_SHAPE, "single-node tree has no environment to close");
  // E_{u->v} into workspace (scratch env set), then dot with E_{v->u}
  const int u = node, v = t->nb[node][0];
  const int ct = ctype_of(compute);
  if (!dtype_ok(envs->dt, compute)) return fail(ctx, TTN_E_DTYPE, "tensor dtype does not match the compute dtype");
  ttn_envs scratch = *envs;
  const int64_t se = envs->slot_elems(u, v);
  const size_t scratch_bytes = (size_t)se * n_pairs * esize(ct);
  const size_t off = (scratch_bytes + 255) / 256 * 256;
  if (off >= ctx->ws_bytes) return fail(ctx, TTN_E_WORKSPACE, "workspace too small for closure scratch");
  ctx->ws_last_plan = nullptr;
  scratch.slot[ttn_envs::dslot(t, u, v)] = ctx->ws;  // scratch at the start of the workspace
  Net net;
  std::string why;
  if (!build_env_net(t, op, bra, ket, &scratch, u, v, net, why)) return fail(ctx, TTN_E_SHAPE, why);
  ttn_status code = TTN_OK;
  Plan* P = get_plan(ctx, net, ct, n_pairs, code);
  if (!P) return code;
  const int kap = (int)t->nb[u].size();
  std::vector<OpAddr> in;
  std::vector<int64_t> ne;
  OpAddr a;
  a.base = bra->ptr[u];
  a.tab = pair_bra;
  a.tab_max = bra->k;
  a.bstride = bra->size[u];
  in.push_back(a);
  ne.push_back(bra->size[u]);
  if (op) {
    OpAddr w;
    w.base = op->W[u];
    w.shared = true;
    in.push_back(w);
    ne.push_back(w_elems(t, op, u));
  }
  OpAddr k;
  k.base = ket->ptr[u];
  k.tab = pair_ket;
  k.tab_max = ket->k;
  k.bstride = ket->size[u];
  in.push_back(k);
  ne.push_back(ket->size[u]);
  for (int i = 1; i < kap; ++i) {
    const int c = t->nb[u][i];
    if (!envs->slot[ttn_envs::dslot(t, c, u)]) return fail(ctx, TTN_E_ARG, "missing incoming environment");
    OpAddr e;
    e.base = envs->slot[ttn_envs::dslot(t, c, u)];
    e.bstride = envs->slot_elems(c, u);
    in.push_back(e);
    ne.push_back(envs->slot_elems(c, u));
  }
  OpAddr o;
  o.base = ctx->ws;
  o.bstride = se;
  ttn_status r = exec_plan(ctx, *P, ct, in, o, Epilogue(), n_pairs, ne, se, off);
  if (r != TTN_OK) return r;
  const void* Ev = envs->slot[ttn_envs::dslot(t, v, u)];
  if (!Ev) return fail(ctx, TTN_E_ARG, "missing incoming environment");
  for (int z0 = 0; z0 < n_pairs; z0 += 65535) {
    const int nz = std::min(65535, n_pairs - z0);
    hipError_t he = launch_batched_dot(stype(ct), (const char*)Ev, nullptr, se, (const char*)ctx->ws + (size_t)z0 * se * esize(ct),
                                       se, se, nz, z0, out, ctx->stream);
    if (he != hipSuccess) return fail(ctx, TTN_E_LAUNCH, hipGetErrorString(he));
  }
  return TTN_OK;
}

ttn_status heff_apply_block(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_envs* envs, int32_t node,
                            int32_t k, const int32_t* pair_ids, const int32_t* x_ids, const double* shift,
                            const double* alpha, const void* X, int32_t x_rows, void* Y, uint32_t flags,
                            ttn_dtype compute) {
  const bool probe = ctx && op && !(flags & TTN_HEFF_DIAG) && k > 0 &&
                     std::find(ctx->probe_nodes.begin(), ctx->probe_nodes.end(), node) != ctx->probe_nodes.end();
  ttn_ctx::CallRec rec;
  const double f0 = ctx ? ctx->flops_done : 0.0;
  if (probe && hipEventCreate(&rec.a) == hipSuccess && hipEventCreate(&rec.b) == hipSuccess)
    (void)hipEventRecord(rec.a, ctx->stream);
  const ttn_status r = ttn::heff_apply_rows(ctx, t, op, envs, node, k, pair_ids, x_ids, nullptr, k, shift, alpha, X,
                                            x_rows, Y, flags, compute);
  if (rec.b) {
    (void)hipEventRecord(rec.b, ctx->stream);
    rec.flops = ctx->flops_done - f0;
    ctx->calls.push_back(rec);
  } else if (rec.a) {
    (void)hipEventDestroy(rec.a);
  }
  return r;
}

}  // extern "C"

namespace ttn {
bool leaf_heff_fusable(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_envs* envs, int u, int ct,
                       LeafHeffArgs& la) {
  if (!op || t->nb[u].size() != 1 || t->phys[u] <= 1 || !(ct == 0 || ct == 1) || !ctx->leg_tabs.empty()) return false;
  const char* fe = getenv("TTN_FUSED_LEAF");
  if (fe && fe[0] == '0') return false;
  const int c = t->nb[u][0];
  la.Db = envs->eb(c, u);
  la.M = envs->em(c, u);
  la.Da = envs->ea(c, u);
  la.d = t->phys[u];
  if (la.M != op->bond(u, c) || leaf_heff_lds_bytes(la.Db, la.M, la.Da, la.d, ct == 0 ? 8 : 4) > LEAF_HEFF_LDS_MAX)
    return false;
  la.E = envs->slot[ttn_envs::dslot(t, c, u)];
  la.e_stride = envs->slot_elems(c, u);
  la.W = op->W[u];
  return true;
}

ttn_status heff_apply_rows(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_envs* envs, int32_t node,
                           int32_t k, const int32_t* pair_ids, const int32_t* x_ids, const int32_t* y_ids,
                           int32_t y_rows, const double* shift, const double* alpha, const void* X, int32_t x_rows,
                           void* Y, uint32_t flags, ttn_dtype compute) {
  if (!ctx || !t || !envs || !Y) return fail(ctx, TTN_E_ARG, "null argument");
  if (node < 0 || node >= t->n) return fail(ctx, TTN_E_ARG, "bad node");
  if (k < 0) return fail(ctx, TTN_E_ARG, "negative k");
  if (flags & ~(TTN_HEFF_NO_SHIFT | TTN_HEFF_DIAG | TTN_HEFF_ACCUM)) return fail(ctx, TTN_E_ARG, "unknown flag");
  if (!(flags & TTN_HEFF_DIAG) && !X) return fail(ctx, TTN_E_ARG, "X is null");
  if (envs->t != t || (op && op->t != t)) return fail(ctx, TTN_E_ARG, "tree mismatch");
  if (!dtype_ok(envs->dt, compute) || (op && !dtype_ok(op->dt, compute)))
    return fail(ctx, TTN_E_DTYPE, "tensor dtype does not match the compute dtype");
  if ((op == nullptr) != envs->identity) return fail(ctx, TTN_E_ARG, "operator / environment kind mismatch");
  if (!pair_ids && k > envs->n_slots) return fail(ctx, TTN_E_ARG, "k exceeds the env slots");
  if (!y_ids && k > y_rows) return fail(ctx, TTN_E_ARG, "Y has fewer rows than the states");
  if (!(flags & TTN_HEFF_DIAG) && (x_rows < 1 || (!x_ids && k > x_rows)))
    return fail(ctx, TTN_E_ARG, "X has fewer rows than the states addressed");
  if (k == 0) return TTN_OK;
  const int u = node;
  if (t->nb[u].empty()) return fail(ctx, TTN_E_SHAPE, "single-node tree");
  for (int c : t->nb[u])
    if (!envs->slot[ttn_envs::dslot(t, c, u)]) return fail(ctx, TTN_E_ARG, "missing incoming environment");
  const int ct = ctype_of(compute);
  const int kap = (int)t->nb[u].size();
  int64_t n_loc = t->phys[u];
  for (int c : t->nb[u]) n_loc *= envs->eb(c, u);
  int64_t n_in = t->phys[u];
  for (int c : t->nb[u]) n_in *= envs->ea(c, u);
  if (flags & TTN_HEFF_DIAG) {
    if (!op) return fail(ctx, TTN_E_ARG, "DIAG needs the operator");
    for (int c : t->nb[u])
      if (envs->eb(c, u) != envs->ea(c, u)) return fail(ctx, TTN_E_SHAPE, "DIAG needs square environments");
    // gather diagonals into the workspace, then contract the small network
    // Wd[w..., p] (shared) and Ed_i[z][b_i, w_i] (batched)
    const int cd = ct == 3 ? 0 : ct;  // the diagonal is gathered and contracted at the storage precision
    const size_t es = esize(cd);
    int64_t wd_elems = t->phys[u];
    for (int c : t->nb[u]) wd_elems *= op->bond(u, c);
    std::vector<int64_t> ed_off(kap);
    int64_t off = (wd_elems + 63) / 64 * 64;
    for (int i = 0; i < kap; ++i) {
      const int c = t->nb[u][i];
      ed_off[i] = off;
      off += ((int64_t)envs->eb(c, u) * envs->em(c, u) * k + 63) / 64 * 64;
    }
    const size_t gather_bytes = (size_t)off * es;
    if (gather_bytes >= ctx->ws_bytes) return fail(ctx, TTN_E_WORKSPACE, "workspace too small for DIAG");
    DiagDesc dd;
    dd.kappa = kap;
    dd.d = t->phys[u];
    dd.W = op->W[u];
    dd.pair = pair_ids;
    dd.n_slots = envs->n_slots;
    dd.flag = ctx->d_flag;
    for (int i = 0; i < kap; ++i) {
      const int c = t->nb[u][i];
      dd.dB[i] = envs->eb(c, u);
      dd.dM[i] = envs->em(c, u);
      dd.dA[i] = envs->ea(c, u);
      dd.E[i] = envs->slot[ttn_envs::dslot(t, c, u)];
      dd.Estride[i] = envs->slot_elems(c, u);
    }
    ctx->ws_last_plan = nullptr;
    hipError_t he = launch_diag_gather(cd, dd, ctx->ws, ed_off.data(), k, ctx->stream);
    if (he != hipSuccess) return fail(ctx, TTN_E_LAUNCH, hipGetErrorString(he));
    Net net;
    std::vector<int> wl, wd, yl, yd;
    for (int i = 0; i < kap; ++i) {
      const int c = t->nb[u][i];
      wl.push_back(3 * i + 1);
      wd.push_back(op->bond(u, c));
      yl.push_back(3 * i);
      yd.push_back(envs->eb(c, u));
    }
    wl.push_back(3 * kap);
    wd.push_back(t->phys[u]);
    yl.push_back(3 * kap);
    yd.push_back(t->phys[u]);
    add_tensor(net.in, wl, wd, 0, net.dims);
    std::ostringstream key;
    key << "diag:" << u;
    for (int i = 0; i < kap; ++i) {
      const int c = t->nb[u][i];
      std::vector<int> el{3 * i, 3 * i + 1};
      std::vector<int> ed{envs->eb(c, u), envs->em(c, u)};
      add_tensor(net.in, el, ed, 1, net.dims);
      key << ":" << ed[0] << "x" << ed[1];
    }
    key << ":d" << t->phys[u];
    net.key = key.str();
    out_layout(yl, yd, net.out_lab, net.out_str);
    ttn_status code = TTN_OK;
    Plan* P = get_plan(ctx, net, cd == 2 ? 1 : cd, k, code);
    if (!P) return code;
    std::vector<OpAddr> in;
    std::vector<int64_t> ne;
    OpAddr w;
    w.base = ctx->ws;
    w.shared = true;
    in.push_back(w);
    ne.push_back(wd_elems);
    for (int i = 0; i < kap; ++i) {
      const int c = t->nb[u][i];
      OpAddr e;
      e.base = (char*)ctx->ws + ed_off[i] * es;
      e.bstride = (int64_t)envs->eb(c, u) * envs->em(c, u);
      in.push_back(e);
      ne.push_back(e.bstride);
    }
    OpAddr o;
    o.base = Y;
    o.bstride = n_loc;
    o.tab = y_ids;
    o.tab_max = y_rows;
    Epilogue ep;
    ep.alpha = nullptr;
    ep.shift = (flags & TTN_HEFF_NO_SHIFT) ? nullptr : shift;
    ep.shift_const = true;
    ep.accum = flags & TTN_HEFF_ACCUM;
    return exec_plan(ctx, *P, cd == 2 ? 1 : cd, in, o, ep, k, ne, n_loc, (gather_bytes + 255) / 256 * 256);
  }
  {
    // identity operator at a three-leg node without a physical leg, FP32, plain
    // output (no shift, scale or accumulation), environment slot = item, output
    // row = item, bonds <= 32: the fused kernel
    bool fuse = !op && kap == 3 && t->phys[u] == 1 && (ct == 1 || ct == 2) && envs->dt == TTN_F32 && !pair_ids &&
                !y_ids && !alpha && !(flags & TTN_HEFF_ACCUM) && ((flags & TTN_HEFF_NO_SHIFT) || !shift);
    const char* fe = getenv("TTN_FUSED_IENV");
    if (fe && fe[0] == '0') fuse = false;
    IHeff3Args fa;
    for (int i = 0; i < 3 && fuse; ++i) {
      const int c = t->nb[u][i];
      fa.dim[i] = envs->eb(c, u);
      fuse = fa.dim[i] == envs->ea(c, u) && fa.dim[i] >= 1 && fa.dim[i] <= 32;
      fa.E[i] = (const float*)envs->slot[ttn_envs::dslot(t, c, u)];
      fa.e_stride[i] = envs->slot_elems(c, u);
    }
    if (fuse) fuse = ienv3_lds_bytes(fa.dim[0], fa.dim[1], fa.dim[2]) <= IENV3_LDS_MAX;
    if (fuse) {
      fa.X = (const float*)X;
      fa.x_size = n_in;
      fa.x_ids = x_ids;
      fa.x_rows = x_rows;
      fa.Y = (float*)Y;
      fa.y_stride = n_loc;
      fa.n = k;
      fa.flag = ctx->d_flag;
      const double D0 = fa.dim[0], D1 = fa.dim[1], D2 = fa.dim[2];
      const double per = 2.0 * D0 * D1 * D2 * (D0 + D1 + D2);
      ctx->flops_done += per * k;
      std::ostringstream key;
      key << "iheff:" << u;
      const std::string ks = key.str();
      // compulsory bytes: X row and Y row, three environments per item
      const double bytes = 4.0 * k * (2.0 * D0 * D1 * D2 + D0 * D0 + D1 * D1 + D2 * D2);
      ttn_prof_rec* pr = prof_begin(ctx, ks.c_str(), "iheff3_kernel", per * k, bytes, k);
      hipError_t he = launch_iheff3(fa, ctx->stream);
      prof_end(ctx, pr);
      if (he != hipSuccess) return fail(ctx, TTN_E_LAUNCH, std::string("fused identity H_eff: ") + hipGetErrorString(he));
      return TTN_OK;
    }
  }
  if (!(flags & TTN_HEFF_NO_SHIFT) && shift && n_in != n_loc)
    return fail(ctx, TTN_E_SHAPE, "a shift needs equal bra and ket bonds");
  {
    // operator product at a node with one virtual leg and a physical leg,
    // FP64 or FP32 arithmetic on its own storage: the fused kernel
    LeafHeffArgs la;
    const bool fuse = kap == 1 && leaf_heff_fusable(ctx, t, op, envs, u, ct, la);
    if (fuse) {
      la.X = X;
      la.x_stride = n_in;
      la.x_ids = x_ids;
      la.x_rows = x_ids ? x_rows : k;
      la.pair_ids = pair_ids;
      la.n_slots = pair_ids ? envs->n_slots : k;
      la.Y = Y;
      la.y_stride = n_loc;
      la.y_ids = y_ids;
      la.y_rows = y_ids ? y_rows : k;
      la.shift = (flags & TTN_HEFF_NO_SHIFT) ? nullptr : shift;
      la.alpha = alpha;
      la.accum = (flags & TTN_HEFF_ACCUM) ? 1 : 0;
      la.n = k;
      la.flag = ctx->d_flag;
      la.gate = ctx->gate;
      const double Db = la.Db, Mw = la.M, Da = la.Da, d = la.d;
      const double per = 2.0 * (Db * Mw * Da * d + Db * d * Mw * d);
      ctx->flops_done += per * k;
      const size_t es = ct == 0 ? 8 : 4;
      // compulsory bytes: X row, Y row and one environment per item, W once
      const double bytes = (double)es * (k * (Da * d + Db * d + Db * Mw * Da) + Mw * d * d);
      std::ostringstream key;
      key << "heff:" << u << ":1:leaf";
      const std::string ks = key.str();
      ttn_prof_rec* pr = prof_begin(ctx, ks.c_str(), "leaf_heff_kernel", per * k, bytes, k);
      hipError_t he = launch_leaf_heff(ct, la, ctx->stream);
      prof_end(ctx, pr);
      if (he != hipSuccess) return fail(ctx, TTN_E_LAUNCH, std::string("fused leaf H_eff: ") + hipGetErrorString(he));
      return TTN_OK;
    }
  }
  Net net;
  std::string why;
  if (!build_heff_net(t, op, envs, u, net, why)) return fail(ctx, TTN_E_SHAPE, why);
  ttn_status code = TTN_OK;
  Plan* P = get_plan(ctx, net, ct, k, code);
  if (!P) return code;
  std::vector<OpAddr> in;
  std::vector<int64_t> ne;
  OpAddr x;
  x.base = X;
  x.tab = x_ids;
  x.tab_max = x_rows;
  x.bstride = n_in;
  in.push_back(x);
  ne.push_back(n_in);
  if (op) {
    OpAddr w;
    w.base = op->W[u];
    w.shared = true;
    in.push_back(w);
    ne.push_back(w_elems(t, op, u));
  }
  const bool per_leg = (int)ctx->leg_tabs.size() == kap;
  for (int i = 0; i < kap; ++i) {
    const int c = t->nb[u][i];
    OpAddr e;
    e.base = envs->slot[ttn_envs::dslot(t, c, u)];
    e.tab = per_leg ? ctx->leg_tabs[i].first : pair_ids;
    e.tab_max = per_leg ? ctx->leg_tabs[i].second : envs->n_slots;
    e.bstride = envs->slot_elems(c, u);
    in.push_back(e);
    ne.push_back(envs->slot_elems(c, u));
  }
  OpAddr o;
  o.base = Y;
  o.bstride = n_loc;
  o.tab = y_ids;
  o.tab_max = y_rows;
  Epilogue ep;
  ep.alpha = alpha;
  if (!(flags & TTN_HEFF_NO_SHIFT) && shift) {
    ep.shift = shift;
    ep.D = x;
  }
  ep.accum = flags & TTN_HEFF_ACCUM;
  return exec_plan(ctx, *P, ct, in, o, ep, k, ne, n_loc);
}

}  // namespace ttn

extern "C" {

// ================================================================== profiling

ttn_status ttn_ctx_flops(ttn_ctx* ctx, double* total, int32_t reset) {
  if (!ctx || !total) return fail(ctx, TTN_E_ARG, "null argument");
  *total = ctx->flops_done;
  if (reset) ctx->flops_done = 0;
  return TTN_OK;
}

}  // extern "C"

namespace ttn {
ttn_prof_rec* prof_begin(ttn_ctx* ctx, const char* key, const char* kernel, double flops, double bytes, int nz) {
  if (!ctx || !ctx->profile || ctx->prof.size() >= 200000 || !prof_selected(ctx, key)) return nullptr;
  ctx->prof.emplace_back();
  ttn_prof_rec* rec = &ctx->prof.back();
  rec->key = key;
  rec->kernel = kernel;
  rec->flops = flops;
  rec->bytes = bytes;
  rec->nz = nz;
  if (hipEventCreate(&rec->a) != hipSuccess || hipEventCreate(&rec->b) != hipSuccess) {
    ctx->prof.pop_back();
    return nullptr;
  }
  (void)hipEventRecord(rec->a, ctx->stream);
  return rec;
}
void prof_end(ttn_ctx* ctx, ttn_prof_rec* rec) {
  if (rec) (void)hipEventRecord(rec->b, ctx->stream);
}
}  // namespace ttn

extern "C" {

ttn_status ttn_ctx_autotune(ttn_ctx* ctx, int32_t on, char* buf, int64_t cap, int64_t* needed) {
  if (!ctx) return fail(nullptr, TTN_E_ARG, "null context");
  if (on >= 0) ctx->autotune = on != 0;
  if (needed) {
    *needed = (int64_t)ctx->tune_log.size() + 1;
    if (buf && cap >= *needed) std::memcpy(buf, ctx->tune_log.c_str(), ctx->tune_log.size() + 1);
  }
  return TTN_OK;
}

ttn_status ttn_ctx_profile(ttn_ctx* ctx, int32_t on) {
  if (!ctx) return fail(nullptr, TTN_E_ARG, "null context");
  ctx->profile = on != 0;
  return TTN_OK;
}

ttn_status ttn_ctx_profile_filter(ttn_ctx* ctx, int32_t n, const char* const* prefixes) {
  if (!ctx || n < 0 || (n > 0 && !prefixes)) return fail(ctx, TTN_E_ARG, "bad filter");
  ctx->prof_filter.clear();
  for (int i = 0; i < n; ++i) {
    if (!prefixes[i]) return fail(ctx, TTN_E_ARG, "null prefix");
    ctx->prof_filter.emplace_back(prefixes[i]);
  }
  return TTN_OK;
}

ttn_status ttn_ctx_probe_heff(ttn_ctx* ctx, int32_t n, const int32_t* nodes) {
  if (!ctx || n < 0 || (n > 0 && !nodes)) return fail(ctx, TTN_E_ARG, "bad probe nodes");
  ctx->probe_nodes.assign(nodes, nodes + n);
  return TTN_OK;
}

ttn_status ttn_ctx_probe_report(ttn_ctx* ctx, int64_t* calls, double* flops, double* ms) {
  if (!ctx || !calls || !flops || !ms) return fail(ctx, TTN_E_ARG, "null argument");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  double f = 0, t = 0;
  for (auto& c : ctx->calls) {
    float e = 0;
    if (hipEventElapsedTime(&e, c.a, c.b) == hipSuccess) t += e;
    f += c.flops;
    (void)hipEventDestroy(c.a);
    (void)hipEventDestroy(c.b);
  }
  *calls = (int64_t)ctx->calls.size();
  *flops = f;
  *ms = t;
  ctx->calls.clear();
  return TTN_OK;
}

ttn_status ttn_ctx_profile_report(ttn_ctx* ctx, char* buf, int64_t cap, int64_t* needed) {
  if (!ctx || !needed) return fail(ctx, TTN_E_ARG, "null argument");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  struct Agg {
    std::string kernel;
    int64_t count = 0;
    double ms = 0, flops = 0, bytes = 0;
    int M = 0, N = 0, K = 0;
    int64_t nz = 0;
  };
  std::map<std::pair<std::string, int>, Agg> agg;
  for (auto& r : ctx->prof) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = 0;
    Agg& a = agg[{r.key, r.step}];
    a.kernel = r.kernel;
    a.count += 1;
    a.ms += ms;
    a.flops += r.flops;
    a.bytes += r.bytes;
    a.M = r.M;
    a.N = r.N;
    a.K = r.K;
    a.nz += r.nz;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  ctx->prof.clear();
  std::ostringstream o;
  for (auto& kv : agg)
    o << kv.first.first << "|" << kv.first.second << "|" << kv.second.kernel << "|" << kv.second.count << "|"
      << kv.second.ms << "|" << kv.second.flops << "|" << kv.second.M << "|" << kv.second.N << "|" << kv.second.K
      << "|" << kv.second.nz << "|" << kv.second.bytes << "\n";
  ctx->prof_text += o.str();
  const std::string& s = ctx->prof_text;
  *needed = (int64_t)s.size() + 1;
  if (buf && cap >= *needed) {
    std::memcpy(buf, s.c_str(), s.size() + 1);
    ctx->prof_text.clear();
  }
  return TTN_OK;
}

// ================================================================== flop counts

ttn_status ttn_flops_heff(const ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_envs* envs, int32_t node,
                          int32_t k, double* flops) {
  (void)ctx;
  if (!t || !envs || !flops || node < 0 || node >= t->n) return fail(nullptr, TTN_E_ARG, "bad arguments");
  Net net;
  std::string why;
  if (!build_heff_net(t, op, envs, node, net, why)) return fail(nullptr, TTN_E_SHAPE, why);
  *flops = min_flops(net.in, net.dims, net.out_lab, k);
  return TTN_OK;
}

ttn_status ttn_flops_env(const ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_block* bra,
                         const ttn_block* ket, int32_t node, int32_t toward, double* fpp) {
  (void)ctx;
  if (!t || !bra || !ket || !fpp || node < 0 || node >= t->n || t->leg_of(node, toward) < 0)
    return fail(nullptr, TTN_E_ARG, "bad arguments");
  // environment bonds follow the blocks
  ttn_envs e;
  e.t = t;
  e.n_slots = 1;
  e.Db = bra->D;
  e.Da = ket->D;
  e.identity = op == nullptr;
  e.M = op ? op->M : std::vector<int>(t->n, 1);
  e.slot.assign(2 * t->n, nullptr);
  Net net;
  std::string why;
  if (!build_env_net(t, op, bra, ket, &e, node, toward, net, why)) return fail(nullptr, TTN_E_SHAPE, why);
  *fpp = min_flops(net.in, net.dims, net.out_lab, 1.0);
  return TTN_OK;
}

}  // extern "C"
