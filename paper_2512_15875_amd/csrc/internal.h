// Internal declarations of the TTN library (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ttn.h"

namespace ttn {

struct Status {
  ttn_status code = TTN_OK;
  std::string msg;
};

// ------------------------------------------------------------------ kernels (gemm.hip)

// One operand of a contraction stage, addressed per batch item z as
//   base + (tab ? tab[z0 + z] : (shared ? 0 : z0 + z)) * bstride + row_off[r] + col_off[c].
struct OpAddr {
  const void* base = nullptr;
  const int32_t* tab = nullptr;  // device batch-index table (may be null)
  int64_t bstride = 0;
  bool shared = false;           // same tensor for every batch item
  bool local = false;            // workspace intermediate: index by z (chunk-local)
  int tab_max = 0;               // number of valid entries a table index may address
};

struct GemmDesc {
  int M = 0, N = 0, K = 0;
  const int32_t* a_om = nullptr;  // [M]
  const int32_t* a_ok = nullptr;  // [K]
  const int32_t* b_ok = nullptr;  // [K]
  const int32_t* b_on = nullptr;  // [N]
  const int32_t* c_om = nullptr;  // [M]
  const int32_t* c_on = nullptr;  // [N]
  bool a_mfast = false, b_nfast = true;
  bool c_mfast = false;  // the output's unit-stride label is a row label (lanes should run along rows)
  int tile = 0;                   // tile configuration id (8: split-K skinny kernel, 9: narrow kernel,
                                  // 10..16: unit-stride-k tiles)
  // host facts about the tables, for the split-K skinny kernel: k offsets are
  // exactly k (a_ok[k] == k, b_ok[k] == k) and every row (column) offset of A
  // (B) is a multiple of 4 elements
  bool k_unit = false;
  bool rows_al4 = false;
};

// the split-K skinny kernel (tile 8) applies: M, N <= 32, long unit-stride k (K % 4 == 0)
inline bool splitk_eligible(const GemmDesc& g, int ctype) {
  return (ctype == 1 || ctype == 2) && g.M <= 32 && g.N <= 32 && g.K >= 64 && g.K % 4 == 0 && !g.a_mfast && !g.b_nfast &&
         g.k_unit && g.rows_al4;
}

// the narrow kernel (tile 9) applies: tall M, N <= 32, short unit-stride k (K <= 32, K % 4 == 0)
inline bool narrow_eligible(const GemmDesc& g, int ctype) {
  return (ctype == 1 || ctype == 2) && g.M >= 64 && g.N <= 32 && g.K <= 32 && g.K % 4 == 0 && !g.a_mfast && !g.b_nfast &&
         g.k_unit && g.rows_al4;
}

// the unit-stride-k tile kernel (tiles 10..16) applies: FP32, both operands
// contiguous along k (K % 4 == 0), row / column offsets multiples of 4
inline bool tn_eligible(const GemmDesc& g, int ctype) {
  return (ctype == 1 || ctype == 3) && g.K >= 32 && g.K % 4 == 0 && !g.a_mfast && !g.b_nfast && g.k_unit &&
         g.rows_al4;
}

struct Epilogue {
  const double* alpha = nullptr;  // per batch item (indexed by z0+z), null = 1
  const double* shift = nullptr;  // per batch item, null = 0; adds -alpha*shift*D
  OpAddr D;                       // addend with C's offsets (base null = none)
  bool accum = false;
  bool shift_const = false;       // subtract alpha*shift (no D read)
};

// dtype: 0 f64, 1 f32 storage with f32 MFMA, 2 f32 storage with bf16 MFMA, 3 f64 storage with f32 MFMA
// gate: null, or a device word; the kernels return at once when it reads zero
hipError_t launch_gemm(int ctype, const GemmDesc& g, const OpAddr& A, const OpAddr& B, const OpAddr& C,
                       const Epilogue& ep, int z0, int nz, int* flag, hipStream_t s, const int32_t* gate = nullptr);

std::string gemm_kernel_name(int ctype, const GemmDesc& g);

hipError_t launch_batched_dot(int ctype, const void* X, const int32_t* xtab, int64_t xstride, const void* Y,
                              int64_t ystride, int64_t n, int nz, int z0, double* out, hipStream_t s);

// fused identity environment of a three-leg node without a physical leg (ienv.hip)
struct IEnv3Args {
  const float* bra = nullptr;  // bra block node tensors [bra_rows][D0][D1][D2]
  const float* ket = nullptr;  // ket block node tensors [ket_rows][D0][D1][D2]
  int64_t bra_size = 0, ket_size = 0;
  const int32_t* pb = nullptr;  // pair -> bra state
  const int32_t* pk = nullptr;  // pair -> ket state
  int bra_rows = 0, ket_rows = 0;
  const float* Ep = nullptr;  // incoming environment of leg p, slot = pair
  const float* Eq = nullptr;  // incoming environment of leg q
  float* Eo = nullptr;        // outgoing environment of leg o
  int64_t ep_stride = 0, eq_stride = 0, eo_stride = 0;
  int dim[3] = {0, 0, 0};     // leg dims (bra == ket)
  int stride[3] = {0, 0, 0};  // leg strides in the node tensor
  int o = 0, p = 1, q = 2;    // output leg, the two contracted legs (p < q)
  int n = 0;                  // pairs
  int* flag = nullptr;
};
struct IHeff3Args {
  const float* X = nullptr;      // block node tensors [x_rows][D0][D1][D2]
  int64_t x_size = 0;
  const int32_t* x_ids = nullptr;  // item -> X row (null: the item index)
  int x_rows = 0;
  const float* E[3] = {nullptr, nullptr, nullptr};  // incoming environments per leg, slot = item
  int64_t e_stride[3] = {0, 0, 0};
  float* Y = nullptr;            // output rows [n][D0][D1][D2]
  int64_t y_stride = 0;
  int dim[3] = {0, 0, 0};
  int n = 0;
  int* flag = nullptr;
};
#define IENV3_LDS_MAX (96 * 1024)
size_t ienv3_lds_bytes(int Do, int Dp, int Dq);
hipError_t launch_ienv3(const IEnv3Args& a, hipStream_t s);
hipError_t launch_iheff3(const IHeff3Args& a, hipStream_t s);

// fused H_eff product at a node with one virtual leg and a physical leg (leaf.hip)
struct LeafHeffArgs {
  const void* X = nullptr;     // [x_rows][Da][d]
  int64_t x_stride = 0;
  const int32_t* x_ids = nullptr;
  int x_rows = 0;
  const void* E = nullptr;     // environment slots [n_slots][Db][M][Da]
  int64_t e_stride = 0;
  const int32_t* pair_ids = nullptr;
  int n_slots = 0;
  const void* W = nullptr;     // [M][d][d] (operator bond, output, input)
  void* Y = nullptr;           // [y_rows][Db][d]
  int64_t y_stride = 0;
  const int32_t* y_ids = nullptr;
  int y_rows = 0;
  const double* shift = nullptr;  // per item (needs Db == Da), null = none
  const double* alpha = nullptr;  // per item, null = 1
  int accum = 0;
  int Db = 0, M = 0, Da = 0, d = 0;
  int n = 0;
  int* flag = nullptr;
  const int32_t* gate = nullptr;  // non-null: return at once when it reads zero
};
#define LEAF_HEFF_LDS_MAX (64 * 1024)
// Whether the fused leaf kernel serves H_eff at node u (one virtual leg, a
// physical leg, FP64 or FP32 arithmetic on its own storage); fills Db, M, Da,
// d, E, e_stride and W of `la` when it does.
bool leaf_heff_fusable(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_envs* envs, int u, int ct,
                       LeafHeffArgs& la);
struct MinresState;
// The whole MINRES local solve of a leaf in one launch (one workgroup per
// state): y holds the warm start on entry and the solution on return, b the
// right-hand side, both [k][n] with n = Da d <= 256; la as for
// launch_leaf_heff with X = Y = y.
hipError_t launch_leaf_minres(int ctype, const LeafHeffArgs& la, const void* b, void* y, int64_t n, double rtol,
                              int maxiter, MinresState* st, hipStream_t s);
size_t leaf_heff_lds_bytes(int Db, int M, int Da, int d, int esize);
// ctype 0: FP64 storage and arithmetic; 1: FP32
hipError_t launch_leaf_heff(int ctype, const LeafHeffArgs& a, hipStream_t s);

// diag(H_eff): out[z][b_N, p] = sum_w Wd[w, p] prod_i Ed_i[z][b_i, w_i] - shift[z]
struct DiagDesc {
  int kappa = 0;
  int dB[4] = {1, 1, 1, 1};       // bra bond per leg
  int dM[4] = {1, 1, 1, 1};       // operator bond per leg
  int dA[4] = {1, 1, 1, 1};       // ket bond per leg (== dB for a diagonal)
  int d = 1;                      // physical dim
  const void* W = nullptr;        // W_u [w..., p, q] (null = identity)
  const void* E[4] = {nullptr, nullptr, nullptr, nullptr};
  const int32_t* pair = nullptr;
  int n_slots = 0;
  int* flag = nullptr;
  int64_t Estride[4] = {0, 0, 0, 0};
};
// Wd[w..., p] = W[w..., p, p] at ws[0..); Ed_i[z][b][w] = E_i[pair(z)][b][w][b] at ws[ed_off[i]..)
hipError_t launch_diag_gather(int ctype, const DiagDesc& dd, void* ws, const int64_t* ed_off, int nz, hipStream_t s);

// per-state scalar recurrence of the batched MINRES (minres.hip)
struct MinresState {
  double beta, c1, s1, c2, s2, phibar, tol;
  int done, iters;
};

// ------------------------------------------------------------------ contraction plans (plan.cpp)

struct Tensor {              // one operand of a network
  std::vector<int> lab;      // index labels in memory order (size-1 legs removed)
  std::vector<int64_t> str;  // element strides
  int batched = 1;           // 0 shared, 1 batched
};

struct Step {
  int a = -1, b = -1;        // operand ids (inputs 0..n_in-1, intermediates n_in..)
  int out = -1;              // intermediate id, or -1 = final output
  GemmDesc g;
  int64_t out_size = 0;      // elements per batch item for an intermediate
  double flops = 0;          // per batch item (or total if both shared)
  bool batched = true;
  int64_t max_a = 0, max_b = 0, max_c = 0;  // largest element offset addressed in A, B, C
  bool tuned = false;        // tile picked by measurement (autotuner)
  // 0: GEMM stage.  1: relayout of a shared input (b == -1): out[k * M + m] =
  // a[a_om[m] + a_ok[k]], so the GEMM after it reads that operand m-fast
  // (or n-fast) and contiguous instead of through strided offsets
  int kind = 0;
};

struct Plan {
  std::string key;
  int n_in = 0;
  std::vector<Step> steps;
  std::vector<int64_t> inter_off;  // workspace offset (elements, per batch item scaled) of each intermediate
  int64_t ws_per_item = 0;         // elements of workspace per batch item
  int64_t ws_shared = 0;           // elements for shared intermediates
  double flops_per_item = 0, flops_shared = 0;
  // every stage table, concatenated on the host (each padded to 16 entries);
  // tab_refs say where each stage's six tables start
  std::vector<int32_t> h_tabs;
  struct TabRef {
    size_t step;
    int which;  // 0 a_om, 1 a_ok, 2 b_ok, 3 b_on, 4 c_om, 5 c_on
    size_t off;
  };
  std::vector<TabRef> tab_refs;
};

// relayout stage: dst[k * M + m] = src[om[m] + ok[k]] (ctype's storage type)
hipError_t launch_relayout(int ctype, const void* src, const int32_t* om, const int32_t* ok, int M, int K, void* dst,
                           hipStream_t s, const int32_t* gate);

// Point a plan's stage descriptors at the device copy of its tables.
void bind_plan_tables(Plan& plan, const int32_t* d_tabs);

// Build the min-flop plan for a network: inputs (with labels/strides), label
// dims, final output labels + strides.  `batch` = number of batch items used
// to weigh batched against shared work.
std::unique_ptr<Plan> make_plan(const std::vector<Tensor>& in, const std::map<int, int>& dims,
                                const std::vector<int>& out_lab, const std::vector<int64_t>& out_str,
                                double batch, int ctype, Status& st);

// Host-to-device upload ordered on `stream` and waited for.  Used instead of
// the legacy synchronous copy, which also waits on the null stream and so
// fails while another thread captures a graph on a blocking stream.
inline bool upload_sync(void* dst, const void* src, size_t bytes, hipStream_t stream) {
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream) == hipSuccess &&
         hipStreamSynchronize(stream) == hipSuccess;
}

// Host-side bounds proof of a plan: every element a stage can address lies in
// its operand (inputs: in_elems per batch item; final output: out_elems).
bool check_plan_bounds(const Plan& P, const std::vector<int64_t>& in_elems, int64_t out_elems, std::string& why);

// minimal flops of a network (same search, no tables)
double min_flops(const std::vector<Tensor>& in, const std::map<int, int>& dims, const std::vector<int>& out_lab,
                 double batch);

}  // namespace ttn

// ------------------------------------------------------------------ handles

struct ttn_ctx;
struct ttn_prof_rec;
namespace ttn {
// heff_apply_block with an output-row table (y_ids[j] = row of Y written by state j)
ttn_status heff_apply_rows(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_envs* envs, int32_t node,
                           int32_t k, const int32_t* pair_ids, const int32_t* x_ids, const int32_t* y_ids,
                           int32_t y_rows, const double* shift, const double* alpha, const void* X, int32_t x_rows,
                           void* Y, uint32_t flags, ttn_dtype compute);
ttn_status api_fail(ttn_ctx* ctx, ttn_status code, const std::string& msg);
// Profiling of a non-contraction launch (QR, Rayleigh-Ritz, MINRES vector
// work): when the context profiles, brackets the launches between begin and
// end with events and records algorithmic flops and compulsory bytes.
::ttn_prof_rec* prof_begin(ttn_ctx* ctx, const char* key, const char* kernel, double flops, double bytes, int nz);
void prof_end(ttn_ctx* ctx, ::ttn_prof_rec* rec);
}  // namespace ttn

struct ttn_tree {
  int n = 0, root = -1;
  std::vector<int> parent, phys;
  std::vector<std::vector<int>> ch, nb;  // children; neighbours [parent, children...]
  int leg_of(int u, int v) const {
    for (size_t i = 0; i < nb[u].size(); ++i)
      if (nb[u][i] == v) return (int)i;
    return -1;
  }
};

struct ttn_ttno {
  const ttn_tree* t = nullptr;
  std::vector<int> M;  // per edge e(u)
  ttn_dtype dt = TTN_F64;
  std::vector<void*> W;
  int bond(int u, int v) const {  // operator bond of edge (u,v)
    return t->parent[u] == v ? M[u] : M[v];
  }
};

struct ttn_block {
  const ttn_tree* t = nullptr;
  int k = 0;
  std::vector<int> D;
  ttn_dtype dt = TTN_F64;
  std::vector<void*> ptr;
  std::vector<int64_t> size;
  int bond(int u, int v) const { return t->parent[u] == v ? D[u] : D[v]; }
  std::vector<int> legdims(int u) const {
    std::vector<int> d;
    for (int v : t->nb[u]) d.push_back(bond(u, v));
    d.push_back(t->phys[u]);
    return d;
  }
};

struct ttn_envs {
  const ttn_tree* t = nullptr;
  int n_slots = 0;
  std::vector<int> Db, M, Da;  // per edge e(u)
  bool identity = false;
  ttn_dtype dt = TTN_F64;
  std::vector<void*> slot;     // 2n directed slots
  static int dslot(const ttn_tree* t, int u, int v) { return t->parent[u] == v ? 2 * u : 2 * v + 1; }
  int eb(int u, int v) const { return t->parent[u] == v ? Db[u] : Db[v]; }
  int em(int u, int v) const { return identity ? 1 : (t->parent[u] == v ? M[u] : M[v]); }
  int ea(int u, int v) const { return t->parent[u] == v ? Da[u] : Da[v]; }
  int64_t slot_elems(int u, int v) const { return (int64_t)eb(u, v) * em(u, v) * ea(u, v); }
};

struct ttn_prof_rec {
  std::string key;     // plan key
  int step = 0;        // stage index in the plan
  std::string kernel;  // kernel instantiation
  double flops = 0;    // algorithmic flops of this launch
  double bytes = 0;    // compulsory bytes of this launch (batched operands once per item, shared ones once)
  int M = 0, N = 0, K = 0, nz = 0;
  hipEvent_t a = nullptr, b = nullptr;
};

struct ttn_ctx {
  bool profile = false;
  // table pool: offset tables of contraction plans, QR row tables and dense
  // GEMM tables are carved from one device allocation made at creation, so no
  // later call allocates device memory; their host copies live as long as the
  // context (the upload is enqueued on the stream without a wait)
  int32_t* pool = nullptr;
  size_t pool_cap = 0, pool_used = 0;  // in int32 entries
  std::deque<std::vector<int32_t>> pool_host;
  // while non-null, every contraction-stage kernel first reads this device
  // word and returns at once when it is zero (the MINRES convergence gate)
  const int32_t* gate = nullptr;
  // reuse of X-independent intermediates across the H_eff applies of one
  // MINRES solve: requested by the MINRES loop (reuse_free), honoured when
  // the same plan with the same inputs ran last on the workspace in one chunk
  bool reuse_free = false;
  const void* ws_last_plan = nullptr;
  std::vector<const void*> ws_last_inputs;
  const void* ws_last_base = nullptr;
  int ws_last_nb = -1;
  // per-leg batch tables of the next H_eff product (leg i = neighbour i of
  // the node): {table, valid entries}; a null table means the identity.  Empty:
  // every leg uses the call's pair_ids (successive randomized compression
  // mixes k-slot and k*chi-slot environments in one product)
  std::vector<std::pair<const int32_t*, int>> leg_tabs;
  // this device's copy of the static scratch array of heff_apply_block_noalloc
  // (looked up at creation; null if the lookup failed)
  void* scratch = nullptr;
  bool autotune = false;  // time every tile shape on a stage's first launch and keep the fastest
  std::string tune_log;   // "plan-key|stage|M|N|K|items|chosen tile|us per tile..." lines
  double flops_done = 0;  // algorithmic contraction flops launched so far
  std::vector<ttn_prof_rec> prof;
  std::string prof_text;  // aggregated, not yet returned
  std::vector<std::string> prof_filter;  // plan-key prefixes the stage profile records (empty: all)
  // call probe: heff_apply_block calls with the operator at these nodes are
  // bracketed by events (whole calls, every stage and gap in between)
  std::vector<int> probe_nodes;
  struct CallRec {
    hipEvent_t a = nullptr, b = nullptr;
    double flops = 0;
  };
  std::vector<CallRec> calls;
  int device = 0;
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
  int* d_flag = nullptr;  // non-finite / not-PD flags
  std::map<std::string, std::unique_ptr<ttn::Plan>> plans;
  std::map<std::string, const int32_t*> tables;  // device offset tables (QR rows etc.), in the pool
};

namespace ttn {
// Every device or pinned-host allocation of the library goes through these
// and is counted (process-wide; ttn_alloc_count).
bool dev_malloc(void** p, size_t bytes);
bool pinned_malloc(void** p, size_t bytes);
// Copy `h` into the context's table pool (256-byte aligned) with an
// asynchronous upload on the context stream; the host copy is kept with the
// context.  Returns null (and sets `code`) when the pool is exhausted.
const int32_t* pool_upload(ttn_ctx* ctx, std::vector<int32_t>&& h, ttn_status& code);
// offsets of the rows of a node tensor with dims `dims` when leg `leg` is the
// column index (a table in the pool, cached per shape); cstride = leg stride
const int32_t* leg_rows_table(ttn_ctx* ctx, const std::vector<int>& dims, int leg, int64_t& cstride, int& m,
                              ttn_status& code);
// whether the stage profile records plans with this key (prefix filter)
bool prof_selected(const ttn_ctx* ctx, const std::string& key);
// the device address of heff_apply_block_noalloc's static scratch array on
// `device` (which must be current); false if it cannot be found
bool noalloc_scratch_setup(int device, void** out);
}  // namespace ttn
