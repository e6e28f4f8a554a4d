/*
 * ttn.h -- C ABI of the MI355X (gfx950) tree-tensor-network eigensolver hot path.
 *
 * Method: Tree Tensor Network Methods for Efficient Calculation of Molecular
 * Vibrational Spectra (arXiv 2512.15875).  A sum-of-products vibrational
 * Hamiltonian (Eq. sum_of_tp) is stored as a tree tensor network operator
 * (TTNO, Eq. ttno) and applied to a block of k tree tensor network states
 * (TTNS, Eq. ttns) inside block LOBPCG (Alg. lobpcg_block) and block inverse
 * iteration (Alg. block_inverse_iteration), whose local problems are the
 * variational-fitting and ALS systems of Sec. II.C.2-3 (Fig. variational,
 * Fig. als).
 *
 * Conventions shared by every call
 * --------------------------------
 * Tree: nodes 0..n-1, parent[u] (-1 at the root), phys[u] (1 for an auxiliary
 *   node).  N(u) = [parent, children in increasing id order].  Edge e(u) joins
 *   non-root u and parent(u).  Directed edges: slot 2u = u -> parent(u),
 *   slot 2u+1 = parent(u) -> u.
 * Layouts: row-major, contiguous, real.
 *   state tensor      A_u[a_N(u)..., p]              (no parent leg at the root)
 *   TTNO tensor       W_u[w_N(u)..., p_out, q_in]
 *   environment u->v  E[slot][b][w][a]  (bra bond, operator bond, ket bond on
 *                     the edge (u,v); the identity operator has w of size 1)
 *   block node buffer [k][size_u]  (all k states of the node, one after another)
 *   local vectors     [k][n_loc] in the node's leg order
 * dtypes: TTN_F64 (double), TTN_F32 (float).  A TTN_BF16 *compute* dtype reads
 *   FP32 tensors, rounds them to bfloat16 on the way into the matrix cores and
 *   accumulates in FP32.
 * Ownership: the caller owns every tensor buffer (device memory) and every
 *   host array it passes; the library keeps pointers to device buffers given
 *   at *_create time and copies host arrays.  The library owns its handles,
 *   contraction plans, the workspace sized at ttn_ctx_create and a 64 MiB
 *   offset-table pool allocated there.  Device (and pinned host) memory is
 *   allocated only by ttn_ctx_create and ttn_sweep_create; ttn_alloc_count
 *   counts those allocations.  Every other call -- the hot-path calls, sweep
 *   steps and sweep runs included -- allocates nothing: a contraction planned
 *   for the first time carves its offset tables from the pool and enqueues
 *   their upload without waiting (the host copy stays with the context), so
 *   the calls can be captured into a HIP graph.
 * Streams: every call enqueues on the context's HIP stream and returns
 *   without synchronising unless stated.
 * Errors: every call returns ttn_status; arguments are validated on the host
 *   before any launch and out-parameters are written only on success; the
 *   message of the last failure is returned by ttn_last_error.  No exception
 *   or abort crosses this boundary.  Host waits: ttn_ctx_sync,
 *   ttn_ctx_set_stream (drains the old stream), ttn_ctx_profile_report, the
 *   autotuner's timed launches, the *_create / *_destroy calls of sweeps and
 *   contexts, and an eager MINRES sweep step, which may wait on an event it
 *   recorded four convergence checks earlier (never under stream capture).
 */
#ifndef TTN_H
#define TTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ttn_status;
enum {
  TTN_OK = 0,
  TTN_E_ARG = 1,        /* null handle, bad index, bad flag */
  TTN_E_SHAPE = 2,      /* tensor dims inconsistent with tree / bonds */
  TTN_E_DTYPE = 3,      /* dtype combination not supported */
  TTN_E_DEVICE = 4,     /* HIP runtime error (message names the call) */
  TTN_E_WORKSPACE = 5,  /* workspace too small even for one state */
  TTN_E_LAUNCH = 6,     /* kernel launch failed */
  TTN_E_NOT_PD = 7,     /* overlap matrix not positive definite and SVQB disabled */
  TTN_E_NONFINITE = 8,  /* NaN/Inf flagged by a kernel (surfaced at ttn_ctx_sync) */
  TTN_E_NOCONV = 9      /* an iterative dense eigensolver did not converge (surfaced at ttn_ctx_sync) */
};

/* TTN_F64_F32 is a compute dtype only: FP64 tensors, FP32 matrix-core
 * arithmetic (operands rounded to FP32 as they are staged, FP32 accumulation,
 * results stored as FP64) -- the inner solves of the mixed-precision local
 * refinement. */
typedef enum { TTN_F64 = 0, TTN_F32 = 1, TTN_BF16 = 2, TTN_F64_F32 = 3 } ttn_dtype;

typedef struct ttn_ctx ttn_ctx;
typedef struct ttn_tree ttn_tree;
typedef struct ttn_ttno ttn_ttno;
typedef struct ttn_block ttn_block;
typedef struct ttn_envs ttn_envs;
typedef struct ttn_sop ttn_sop;

/* ------------------------------------------------------------ housekeeping */

/* Create a context on `device` using HIP stream `hip_stream` (NULL = default
 * stream) with a device workspace of `workspace_bytes` for contraction
 * intermediates (0 = 1 GiB). */
ttn_status ttn_ctx_create(int device, void* hip_stream, size_t workspace_bytes, ttn_ctx** out);
ttn_status ttn_ctx_set_stream(ttn_ctx* ctx, void* hip_stream);
/* Synchronise the context stream; returns TTN_E_NONFINITE if a kernel raised
 * the non-finite flag since the last sync (the flag is then cleared). */
ttn_status ttn_ctx_sync(ttn_ctx* ctx);
ttn_status ttn_ctx_destroy(ttn_ctx* ctx);
const char* ttn_last_error(const ttn_ctx* ctx);
/* Library version string. */
const char* ttn_version(void);
/* Number of device and pinned-host allocations the library has made in this
 * process (ttn_ctx_create: workspace, table pool, flags; ttn_sweep_create:
 * environments, vectors, convergence ring).  A caller checks that a sequence
 * of calls allocates nothing by reading it before and after. */
ttn_status ttn_alloc_count(int64_t* out);

/* Tree (Eq. ttns / Appendix B topologies).  Host arrays are copied. */
ttn_status ttn_tree_create(int32_t n_nodes, const int32_t* parent, const int32_t* phys, ttn_tree** out);
ttn_status ttn_tree_destroy(ttn_tree* t);

/* TTNO (Eq. ttno): per-node device pointers W[u] (layout above, dtype
 * `dtype`), operator bond op_bond[u] for the edge e(u) (entry at the root
 * ignored).  Pointers are borrowed for the handle's lifetime. */
ttn_status ttn_ttno_create(ttn_ctx* ctx, const ttn_tree* t, const int32_t* op_bond, ttn_dtype dtype,
                           void* const* W, ttn_ttno** out);
ttn_status ttn_ttno_destroy(ttn_ttno* o);

/* Block of k states (Eq. ttns, one TTNS per state, all with the bond
 * dimensions bond[u] of edge e(u)).  node_ptr[u] is a device buffer of
 * k * size_u elements of `dtype`.  Borrowed for the handle's lifetime. */
ttn_status ttn_block_create(ttn_ctx* ctx, const ttn_tree* t, int32_t k, const int32_t* bond, ttn_dtype dtype,
                            void* const* node_ptr, ttn_block** out);
ttn_status ttn_block_destroy(ttn_block* b);
/* Number of elements of one state's tensor at node u. */
ttn_status ttn_block_node_size(const ttn_block* b, int32_t u, int64_t* size_out);

/* Environment storage for `n_slots` (bra, ket) pairs: for directed edge slot
 * s (see above) slot_ptr[s] is a device buffer [n_slots][bra_bond][M][ket_bond]
 * of `dtype`, with M = op_bond of the edge or 1 when op_bond is NULL
 * (identity operator).  Unused directed edges may be NULL. */
ttn_status ttn_envs_create(ttn_ctx* ctx, const ttn_tree* t, int32_t n_slots, const int32_t* bra_bond,
                           const int32_t* op_bond, const int32_t* ket_bond, ttn_dtype dtype,
                           void* const* slot_ptr, ttn_envs** out);
ttn_status ttn_envs_destroy(ttn_envs* e);

/* ------------------------------------------------------------ the hot path */

/* Environment update (Sec. II.C.2-3; the shaded blocks of Fig. variational
 * and Fig. als), for every pair p < n_pairs:
 *   E^p_{u->v}[b,w,a] = sum A^{bra[p]}_u[b_N,p] W_u[w_N,p,q] A^{ket[p]}_u[a_N,q]
 *                       prod_{c in N(u)\v} E^p_{c->u}[b_c,w_c,a_c]
 * op NULL = identity operator.  pair_bra / pair_ket: device int32[n_pairs],
 * indices into the bra / ket blocks.  Incoming environments are read from, and
 * the result written to, slot p of `envs`.  u = node, v = toward (a
 * neighbour of u).  compute: TTN_F64 needs F64 tensors; TTN_F32 / TTN_BF16
 * need F32 tensors. */
ttn_status ttno_env_update(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_block* bra,
                           const ttn_block* ket, int32_t n_pairs, const int32_t* pair_bra,
                           const int32_t* pair_ket, int32_t node, int32_t toward, ttn_envs* envs,
                           ttn_dtype compute);

/* Closure (the Gram entries <bra|O|ket> at node u from all incoming
 * environments, Alg. lobpcg_block's H~ and M~):
 *   out[p] = sum A^{bra[p]}_u W_u A^{ket[p]}_u prod_{c in N(u)} E^p_{c->u}
 * out: device double[n_pairs]. */
ttn_status ttno_env_close(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_block* bra,
                          const ttn_block* ket, int32_t n_pairs, const int32_t* pair_bra,
                          const int32_t* pair_ket, int32_t node, const ttn_envs* envs, double* out,
                          ttn_dtype compute);

#define TTN_HEFF_APPLY 0u     /* Y = alpha (H_eff - shift) X                  */
#define TTN_HEFF_NO_SHIFT 1u  /* ignore shift                                  */
#define TTN_HEFF_DIAG 2u      /* Y = diag(H_eff) - shift (X unused)            */
#define TTN_HEFF_ACCUM 4u     /* add into Y instead of overwriting it          */

/* Local effective-Hamiltonian product for k states at node u (Sec. II.C.2-3):
 *   Y_j[b_N,p] = alpha_j * ( sum W_u[w_N,p,q] X_{x(j)}[a_N,q]
 *                prod_{c in N(u)} E^{pair(j)}_{c->u}[b_c,w_c,a_c] - s_j X_{x(j)}[b_N,p] )
 * op NULL = identity operator (the fitting / ALS right-hand side when the
 * environments pair a target with a source state).
 * pair_ids: device int32[k] env slot per state (NULL = j).
 * x_ids:    device int32[k] row of X per state (NULL = j), each < x_rows.
 * shift, alpha: device double[k] (NULL = 0 and 1).
 * X: [x_rows][n_in], Y: [k][n_loc] (device; dtype = the tensors' dtype);
 * n_in / n_loc are the products of the ket / bra bonds times phys[u].
 * Out-of-range pair_ids / x_ids entries are clamped on the device and reported
 * as TTN_E_ARG by the next ttn_ctx_sync.
 * With TTN_HEFF_DIAG, Y_j = diag(H_eff) - s_j (X, x_ids, alpha unused). */
ttn_status heff_apply_block(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_envs* envs,
                            int32_t node, int32_t k, const int32_t* pair_ids, const int32_t* x_ids,
                            const double* shift, const double* alpha, const void* X, int32_t x_rows,
                            void* Y, uint32_t flags, ttn_dtype compute);

/* Rayleigh-Ritz for `batch` independent problems H~ v = lambda S~ v
 * (Alg. lobpcg_block / Alg. block_inverse_iteration), FP64 on the device.
 * H, S: device double[batch][ld][ld] (row-major, symmetric; only m[b] x m[b]
 * used).  m: host int32[batch] (m[b] <= ld <= 512).  Cholesky of S~; when a
 * pivot <= drop_tol * max diag(S~) the problem falls back to SVQB (eigen-
 * decomposition of S~, directions with sigma <= drop_tol * sigma_max dropped).
 * Outputs (device): evals double[batch][nev] ascending; V double[batch][ld][nev]
 * (column j = eigenvector j, V^T S~ V = I, largest-magnitude entry of each
 * column positive); rank_out int32[batch] (m[b] or the SVQB rank).
 * allow_svqb = 0 makes a non-positive-definite S~ an error (TTN_E_NOT_PD,
 * reported at ttn_ctx_sync).  The symmetric eigenproblems are solved by
 * Householder tridiagonalisation and implicit QL; a QL iteration that does not
 * converge is reported as TTN_E_NOCONV at ttn_ctx_sync. */
ttn_status rayleigh_ritz(ttn_ctx* ctx, int32_t batch, const int32_t* m, int32_t ld, const double* H,
                         const double* S, int32_t nev, double drop_tol, int32_t allow_svqb,
                         double* evals, double* V, int32_t* rank_out);

/* heff_apply_block for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, semantics, kernels and error behaviour as
 * heff_apply_block; the contraction intermediates live in a static device
 * array of 256 MiB per device (one state's intermediates must fit in it --
 * TTN_E_WORKSPACE otherwise -- and the states are processed in chunks that
 * fit), found at ttn_ctx_create and kept until the process ends.  The call
 * makes no device or pinned allocation (offset tables of a contraction
 * planned for the first time come from the context's table pool).  Every
 * call on one device shares that device's array: calls that overlap in time
 * on one device (two streams, two contexts or two threads) race. */
ttn_status heff_apply_block_noalloc(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_envs* envs,
                                    int32_t node, int32_t k, const int32_t* pair_ids, const int32_t* x_ids,
                                    const double* shift, const double* alpha, const void* X, int32_t x_rows,
                                    void* Y, uint32_t flags, ttn_dtype compute);

/* ------------------------------------------------------------ sweep (ALS / fitting) */

/* MINRES: local MINRES on (H_eff - s_j); DIAG: y = b / (diag(H_eff) - s_j);
 * FIT: y_u = the fitting sum; SKIP: no local solve (only the centre move, as
 * on the later visits of a node during an Euler tour).
 * LEARNED (the learned local preconditioner; not in the paper, which names
 * better preconditioners as future work in its outlook): the MLP of
 * ttn_mlp_forward maps the tile features of (b, diag(H_eff) - s_j) to a
 * candidate y_L; the DIAG solution y_D stays the fallback and the yardstick: the
 * local result is the minimal-residual combination a y_D + c y_L, y_L the
 * network's correction (2x2 least
 * squares on |(H_eff - s_j)(a y_D + c y_L) - b|, FP64), and c = 0 whenever
 * that system is singular or not finite, so a local step never leaves a
 * larger residual than the DIAG step scaled by its own best factor. */
typedef enum {
  TTN_SOLVE_MINRES = 0,
  TTN_SOLVE_DIAG = 1,
  TTN_SOLVE_FIT = 2,
  TTN_SOLVE_SKIP = 3,
  TTN_SOLVE_LEARNED = 4
} ttn_solve_mode;

/* Start of the local MINRES (mode MINRES): NONE starts from the current y_u
 * (the paper's warm start).  DIAG and LEARNED first correct it: with
 * r0 = b - (H_eff - s_j) y_u, the correction c is the DIAG step r0 / (diag -
 * s_j) at its minimal-residual scale (DIAG), or the LEARNED map applied to
 * r0 in place of b (LEARNED, needs mlp_params); y_u += c and MINRES runs its
 * maxiter iterations from there.  Costs one (DIAG) or two (LEARNED) extra
 * H_eff applications of the k states per local solve.  Not in the paper. */
typedef enum { TTN_WARM_NONE = 0, TTN_WARM_DIAG = 1, TTN_WARM_LEARNED = 2 } ttn_warm_start;

/* Symmetric positive-definite preconditioning of the local MINRES (mode
 * MINRES): with d = diag(H_eff) - s_j of each state, D = |d| (DIAG) or
 * D = sqrt(d^2 + gamma^2) (DAMPED_DIAG, gamma = precond_damp * rms(d)), MINRES
 * runs on D^-1/2 (H_eff - s_j) D^-1/2 z = D^-1/2 b from z = D^1/2 y_u and
 * y_u = D^-1/2 z at the end (split preconditioning: the same Krylov iterates
 * as preconditioned MINRES with M = D; rtol and the reported residual refer
 * to the scaled system).  Costs one diagonal and four element-wise scalings
 * per local solve and two per iteration.  Not in the paper; DAMPED_DIAG's
 * damping is the learned parameter (fitted on training local systems). */
typedef enum { TTN_PRECOND_NONE = 0, TTN_PRECOND_DIAG = 1, TTN_PRECOND_DAMPED_DIAG = 2 } ttn_precond;

typedef struct {
  int32_t mode;              /* ttn_solve_mode */
  int32_t maxiter;           /* MINRES iterations per local solve */
  double rtol;               /* MINRES: stop when |residual| <= rtol * |b| */
  const float* mlp_params;   /* LEARNED: device FP32 parameters (ttn_mlp_num_params() floats) */
  int32_t mlp_compute;       /* LEARNED: TTN_BF16 or TTN_F32 matrix-core arithmetic */
  int32_t refine;            /* MINRES on an FP64 sweep, > 0: mixed-precision iterative refinement with this
                                many steps: r = b - (H_eff - s) y in FP64, c from MINRES with TTN_F64_F32
                                applies (rtol max(rtol, 1e-6), maxiter iterations), y += c in FP64 */
  double* learned_coef;      /* LEARNED, optional: device double[k][2], (a, c) of the last local step */
  int32_t warm;              /* ttn_warm_start; MINRES with refine = 0 only */
  int32_t precond;           /* ttn_precond; MINRES with refine = 0 and warm = NONE only */
  double precond_damp;       /* DAMPED_DIAG: gamma = precond_damp * rms(diag - s_j) of the state */
} ttn_solve_opts;

typedef struct ttn_sweep ttn_sweep;

/* A sweep over a target block y (k states) solving, node by node,
 *   MINRES / DIAG:  (H - s_j) y_j = phi_j           (ALS, Sec. II.C.3)
 *   FIT:            y_t = sum_terms c * O phi_s     (fitting, Sec. II.C.2)
 * Source terms: up to 2 (op_i, block_i, n_i terms (target t, source s,
 * coefficient c)); for MINRES/DIAG exactly one identity-operator term with
 * n = k and targets 0..k-1.  `shift` device double[k] (MINRES/DIAG).
 * H-environments (y,y) use op; RHS environments (y, source) use op_i.
 * The library allocates the environment storage, the RHS scratch and the
 * MINRES vectors at creation.  The target block must be in canonical form
 * with its orthogonality centre at `centre`; ttn_sweep_init computes every
 * environment toward the centre.  compute: TTN_F64 or TTN_F64_F32 for an FP64
 * target (the latter contracts on FP32 matrix cores; storage, environments and
 * the local vectors stay FP64), TTN_F32 or TTN_BF16 for an FP32 target. */
/* term_target / term_source are HOST int32 arrays (copied); term_coef are
 * DEVICE double arrays read at every FIT step (so coefficients may change
 * between sweeps, e.g. the Rayleigh-Ritz vectors of an LOBPCG iteration). */
ttn_status ttn_sweep_create(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, ttn_block* target,
                            int32_t n_src, const ttn_ttno* const* src_op, const ttn_block* const* src_block,
                            const int32_t* n_terms, const int32_t* const* term_target,
                            const int32_t* const* term_source, const double* const* term_coef,
                            const double* shift, ttn_dtype compute, ttn_sweep** out);
ttn_status ttn_sweep_init(ttn_sweep* sw, int32_t centre);
/* Synchronises the sweep's context stream, then frees the sweep.  A sweep
 * keeps a pointer to its context: destroy every sweep before its context. */
ttn_status ttn_sweep_destroy(ttn_sweep* sw);

/* One local step of a sweep at `node` (the current orthogonality centre):
 * local right-hand side from the source environments, local solve (MINRES on
 * (H_eff - s_j), DIAG, or the FIT sum), then, if next >= 0, a QR gauge move
 * of every state toward the neighbour `next` (R absorbed into `next`) and the
 * environment updates across the crossed edge.  iters_out / resid_out:
 * device int32[k] / double[k] MINRES iterations and final residual norm
 * estimates (may be NULL). */
ttn_status sweep_step(ttn_ctx* ctx, ttn_sweep* sw, int32_t node, int32_t next, const ttn_solve_opts* opts,
                      int32_t* iters_out, double* resid_out);

/* QR gauge move of all k states of a block from node u to neighbour v
 * (Sec. II.A.1): A_u reshaped [rest, D_e] = Q R (diag R >= 0), A_u <- Q,
 * A_v <- R contracted into its leg toward u.  FP64 arithmetic. */
ttn_status ttn_block_move_centre(ttn_ctx* ctx, ttn_block* b, int32_t u, int32_t v);

/* Scale state j's tensor at node u by scale[j] (device double[k]). */
ttn_status ttn_block_scale_node(ttn_ctx* ctx, ttn_block* b, int32_t u, const double* scale);

/* Squared norms of the k tensors at node u: out device double[k]. */
ttn_status ttn_block_node_norms2(ttn_ctx* ctx, const ttn_block* b, int32_t u, double* out);

/* Scale each of the k tensors at node u to unit norm (the state's norm when u
 * is its orthogonality centre); norms_out: device double[k] of the norms
 * before scaling (may be NULL). */
ttn_status ttn_block_normalize_node(ttn_ctx* ctx, ttn_block* b, int32_t u, double* norms_out);

/* Symmetric scatter used to assemble Gram matrices from pair values:
 * out[idx_a[i]] = out[idx_b[i]] = vals[i] (all device arrays, linear indices). */
ttn_status ttn_scatter_sym(ttn_ctx* ctx, int32_t n, const int32_t* idx_a, const int32_t* idx_b, const double* vals,
                           double* out);

/* y = alpha * x for device double vectors of length n. */
ttn_status ttn_vec_scale(ttn_ctx* ctx, int32_t n, const double* x, double alpha, double* y);

/* y = sqrt(x) elementwise for device double vectors of length n (the residual
 * norms of Alg. lobpcg_block from their squares). */
ttn_status ttn_vec_sqrt(ttn_ctx* ctx, int32_t n, const double* x, double* y);

/* dst[i] = src[idx[i]] for idx[i] >= 0, else `fill` (device arrays; idx
 * int32[n], src double[src_n], dst double[n]): the recombination coefficients
 * V[l, j] of Alg. lobpcg_block and Alg. block_inverse_iteration laid out in a
 * fitting sweep's term order.  An index >= src_n writes `fill` and is
 * reported as TTN_E_ARG by the next ttn_ctx_sync. */
ttn_status ttn_vec_gather(ttn_ctx* ctx, int32_t n, const int32_t* idx, const double* src, int32_t src_n, double fill,
                          double* dst);

/* Rows [0, rows) of every node tensor of `src` converted into `dst` (same
 * tree structure and bonds; FP32 <-> FP64 or a plain copy): the promotion of a
 * low-precision block to FP64 for refinement. */
ttn_status ttn_block_convert(ttn_ctx* ctx, const ttn_block* src, ttn_block* dst, int32_t rows);

/* ------------------------------------------------------------ successive randomized compression */

/* y_j ~ H x_j for the k states of a block by successive randomized
 * compression (Sec. II.C.1; Eq. matrix random compression, Fig. random
 * tensor, Fig. src), sketch size chi.  The test matrix of the method is a
 * Khatri-Rao product: column l is the product over the physical nodes u of
 * row l of omega[u] (device, [chi][phys_u] in the tensors' dtype; ignored at
 * auxiliary nodes), drawn by the caller.  Steps: the environments of
 * <omega_l|H|x_j> on every edge; then, from the leaves to the root, each
 * non-root node's local sketch (its H and x tensors contracted with the
 * compressed children and with the sketch of everything outside its subtree,
 * one column per l) is QR-factorised (Householder, diag(R) >= 0) and Q becomes
 * y's tensor there -- a node whose local space has at most chi dimensions
 * keeps it whole (identity) -- and finally the root's tensors are contracted
 * with the compressed children.  y comes out canonical at the root.
 * y's bonds must be ttn_src_bonds(tree, chi): edge (u, parent) keeps
 * min(chi, prod of u's children's bonds * phys[u]).  x, y and the operator
 * share one dtype; compute TTN_F64 (FP64) or TTN_F32 (FP32).  ttn_src_create
 * allocates the sketch environments (k * chi slots per directed edge) and the
 * compressed environments; ttn_src_apply allocates nothing. */
typedef struct ttn_src ttn_src;
ttn_status ttn_src_bonds(const ttn_tree* t, int32_t chi, int32_t* bonds_out);
ttn_status ttn_src_create(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_block* x, ttn_block* y,
                          int32_t chi, ttn_dtype compute, ttn_src** out);
ttn_status ttn_src_apply(ttn_ctx* ctx, ttn_src* s, const void* const* omega);
/* Synchronises the context stream, then frees the handle. */
ttn_status ttn_src_destroy(ttn_src* s);

/* ------------------------------------------------------------ bond expansion */

/* Grows the bonds of the k states of x into y (y's bonds >= x's, at most
 * n_sketch larger on every edge, each within its node's local space) keeping
 * every state exactly: the dynamic bond dimensions of variational fitting
 * (Sec. II.C.2: local residual, rank-revealing QR, expansion), applied where
 * the maximum bond grows between the LOBPCG and inverse-iteration stages
 * (Sec. III.B).  From the leaves to the root, at each non-root node u: the
 * local x_u with its children legs in y's bases and its parent leg open is
 * QR-factorised (basis Q_x); the local H x is sketched on the parent leg with
 * n_sketch Khatri-Rao columns (row l of omega[u], device, [n_sketch][phys_u]
 * in the tensors' dtype, drawn by the caller; ignored at auxiliary nodes --
 * the same sketch as ttn_src); a Householder QR of [Q_x | sketch] with Q_x
 * first and unpivoted, then y->D[u] - x->D[u] steps pivoting on the largest
 * remaining column norm (first on ties), gives the new directions (diag(R) >= 0)
 * and y_u = [Q_x, new directions].  The root takes x_root in the children's new
 * bases, so y is canonical at the root and equal to x as a vector.  x, y and
 * the operator share one dtype; compute TTN_F64 or TTN_F32.  ttn_expand_create
 * allocates the sketch environments (k * n_sketch slots per directed edge) and
 * the per-node work buffers; ttn_expand_apply allocates nothing. */
typedef struct ttn_expand ttn_expand;
ttn_status ttn_expand_create(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_block* x, ttn_block* y,
                             int32_t n_sketch, ttn_dtype compute, ttn_expand** out);
ttn_status ttn_expand_apply(ttn_ctx* ctx, ttn_expand* e, const void* const* omega);
/* Synchronises the context stream, then frees the handle. */
ttn_status ttn_expand_destroy(ttn_expand* e);

/* ------------------------------------------------------------ operator compiler (host) */

/* Sum-of-products -> TTNO in FP64 on the host (Sec. II.A.3, Eq. sum_of_tp):
 * H = sum_i omega_i n_i + sum_m coef_m prod (q_i)^{pow}, in the harmonic-
 * oscillator basis of size dims[mode] (exact projections of q^k).
 * mono_ptr[m]..mono_ptr[m+1] index the (mode, power) pairs of monomial m in
 * mono_mode / mono_pow.  node_mode[u]: the mode carried by node u, -1 for an
 * auxiliary node.  Built with a channel automaton and compressed by
 * SVD to the operator Schmidt rank (relative cutoff rel_tol). */
ttn_status ttn_sop_build(const ttn_tree* t, const int32_t* node_mode, int32_t n_modes, const double* omega,
                         const int32_t* dims, int32_t n_mono, const int32_t* mono_ptr,
                         const int32_t* mono_mode, const int32_t* mono_pow, const double* coef,
                         double rel_tol, ttn_sop** out);
/* The same operator from a state diagram (Sec. II.A.3): edges leaves to
 * root, every term (or group of terms merged below) an edge of the bipartite
 * graph between its descriptor inside the subtree (operator at the node and
 * child channels) and its operator string outside; a minimum vertex cover
 * (Konig, from an augmenting-path matching in order of first appearance)
 * gives the channels -- covered descriptors coefficient-free, covered outside
 * strings carrying the summed coefficient x descriptor of their terms, which
 * merge there; terms merged in another branch take coefficient-free channels.
 * No compression: the tensors keep the diagram's sparsity.  Bonds equal the
 * operator Schmidt ranks for terms with generic coefficients; algebraic
 * redundancy between coefficients (e.g. all couplings equal) is not seen.
 * Same arguments as ttn_sop_build without rel_tol. */
ttn_status ttn_sop_build_sd(const ttn_tree* t, const int32_t* node_mode, int32_t n_modes, const double* omega,
                            const int32_t* dims, int32_t n_mono, const int32_t* mono_ptr,
                            const int32_t* mono_mode, const int32_t* mono_pow, const double* coef, ttn_sop** out);
/* op_bond[u] for every edge e(u) (root entry 0). */
ttn_status ttn_sop_bonds(const ttn_sop* s, int32_t* op_bond);
/* Copy node u's tensor (layout W_u above, FP64) into host buffer `out` of
 * `cap` doubles. */
ttn_status ttn_sop_tensor(const ttn_sop* s, int32_t u, double* out, int64_t cap);
ttn_status ttn_sop_destroy(ttn_sop* s);

/* ------------------------------------------------------------ measurement */

/* Per-stage timing: with profiling on, every contraction stage launch is
 * bracketed by HIP events on the context stream.  The report (synchronises
 * the stream, then clears the records) is text, one line per (plan, stage):
 * "plan-key|stage|kernel|launches|total_ms|algorithmic_flops|M|N|K|batch_items|compulsory_bytes"
 * (compulsory bytes: every batched operand read once per item, shared operands
 * once, the output written once and read when accumulating).  `needed`
 * receives the size including the terminating NUL; the text is written to
 * `buf` and then cleared only when cap >= needed (call once with buf NULL to
 * size the buffer). */
ttn_status ttn_ctx_profile(ttn_ctx* ctx, int32_t on);
/* Restrict the stage profile to plans whose key starts with one of the n
 * prefixes (n = 0: every plan).  H_eff plans at node u with the operator have
 * keys starting "heff:<u>:1", environment updates "env:<u>>". */
ttn_status ttn_ctx_profile_filter(ttn_ctx* ctx, int32_t n, const char* const* prefixes);
/* Call probe: every later heff_apply_block call with the operator (not DIAG)
 * at one of the n nodes is bracketed by HIP events on the context stream --
 * the whole call, all its stages and the gaps between them (n = 0: off).
 * ttn_ctx_probe_report synchronises the stream and returns the number of
 * probed calls, their algorithmic flops (the minimum-order count) and the sum
 * of their event times in ms, then clears the records. */
ttn_status ttn_ctx_probe_heff(ttn_ctx* ctx, int32_t n, const int32_t* nodes);
ttn_status ttn_ctx_probe_report(ttn_ctx* ctx, int64_t* calls, double* flops, double* ms);
/* Tile autotuner.  on = 1: the first launch of every contraction stage that
 * overwrites its output runs each tile shape (128x128, 64x64, 128x64,
 * 64x128, 32x64, 64x32, 32x32) twice, times the second run with HIP events (synchronising), and keeps the
 * fastest for the plan; on = 0 stops tuning new stages (tuned choices stay);
 * on < 0 leaves the setting.  The log (one line per tuned stage: "plan-key|
 * stage|M|N|K|items|heuristic->chosen|tile:microseconds...") is copied to buf
 * when cap >= *needed (needed may be NULL).  Tuning never runs under stream
 * capture or profiling. */
ttn_status ttn_ctx_autotune(ttn_ctx* ctx, int32_t on, char* buf, int64_t cap, int64_t* needed);
/* Algorithmic contraction flops (minimum-order counts of every planned
 * contraction launched on this context) since creation or the last reset. */
ttn_status ttn_ctx_flops(ttn_ctx* ctx, double* total, int32_t reset);
ttn_status ttn_ctx_profile_report(ttn_ctx* ctx, char* buf, int64_t cap, int64_t* needed);

/* Sweep executor: n_sweeps sweeps, each a depth-first Euler tour from the
 * root (children in index order) with the node's local solve on its first
 * visit and only centre moves on later visits; init_first = 1 rebuilds every
 * environment toward the root first (ttn_sweep_init).  use_graph = 1 replays
 * the whole sequence as one HIP graph on the context stream: the first call
 * with an option set runs eagerly (building plans and tables), the second
 * captures and launches, later ones replay.  Graphs need a non-null context
 * stream and are skipped under profiling.  A captured MINRES step records all
 * maxiter iterations; every 25 iterations a device count of the unconverged
 * states gates the following iterations' kernels, which return at once when
 * it is zero.  The algorithmic flop counter is advanced by the captured
 * amount on each replay (an upper bound for gated MINRES work).  Every pointer reachable from the
 * sweep (blocks, coefficients, shifts, opts' device arrays, iters/resid) must
 * keep its address between replays. */
ttn_status ttn_sweep_run(ttn_ctx* ctx, ttn_sweep* sw, const ttn_solve_opts* opts, int32_t n_sweeps,
                         int32_t init_first, int32_t use_graph, int32_t* iters, double* resid);

/* ------------------------------------------------------------ learned local preconditioner
 *
 * A 3-layer perceptron 128 -> 256 -> 256 -> 64 with SiLU after the two hidden
 * layers, applied to tiles of T = 64 consecutive entries of a local vector.
 * Parameters: one device FP32 array of ttn_mlp_num_params() floats, row-major
 * W1[128][256], b1[256], W2[256][256], b2[256], W3[256][64], b3[64]; a layer
 * computes out = in W + b.  compute = TTN_BF16 rounds both GEMM operands to
 * bfloat16 as they are staged (FP32 master weights, FP32 accumulation);
 * TTN_F32 keeps FP32 operands.  All pointers are device pointers owned by the
 * caller; every call is asynchronous on the context stream.
 *
 * Features of state j's tile t: [b_tile / |b_j|, (d_tile) / sigma_j] with
 * d = diag(H_eff) - s_j, sigma_j = mean |d| over the node, zero past the
 * vector's end; the network output is the correction to the DIAG step b / d
 * in units of |b_j| / sigma_j (a zero output leaves the DIAG step). */
int64_t ttn_mlp_num_params(void);

/* Y[n][64] = MLP(X[n][128]); acts (nullable): float[4][n][256] receives the
 * pre- and post-activation of both hidden layers for ttn_mlp_backward (null:
 * context workspace, 4 KiB per row, TTN_E_WORKSPACE if too small). */
ttn_status ttn_mlp_forward(ttn_ctx* ctx, const float* params, int32_t n, const float* X, float* Y, float* acts,
                           ttn_dtype compute);
/* grads (ttn_mlp_num_params floats, overwritten) of sum over the rows of
 * <dY, Y> for the forward pass recorded in acts.  Uses 2 KiB of workspace per
 * row. */
ttn_status ttn_mlp_backward(ttn_ctx* ctx, const float* params, int32_t n, const float* X, const float* acts,
                            const float* dY, float* grads, ttn_dtype compute);
/* Mean-squared error over n x 64 outputs: loss (device double, overwritten)
 * and its gradient dY = 2 (Y - T) / (64 n). */
ttn_status ttn_mlp_loss(ttn_ctx* ctx, int32_t n, const float* Y, const float* T, float* dY, double* loss);
/* One Adam step (bias-corrected, step >= 1) on all parameters. */
ttn_status ttn_mlp_adam(ttn_ctx* ctx, float* params, float* m, float* v, const float* grads, float lr, float beta1,
                        float beta2, float eps, int32_t step);
/* Tile features of k local vectors b[k][n] with diagonals d[k][n] (storage
 * TTN_F64 or TTN_F32): X[k * ceil(n/64)][128]; scales double[k][2] receives
 * (|b_j|, sigma_j). */
ttn_status ttn_precond_features(ttn_ctx* ctx, int32_t k, int64_t n, ttn_dtype storage, const void* b, const void* d,
                                double* scales, float* X);
/* Training targets: the correction of the solution tiles y[k][n] over the
 * DIAG step, in network units ((y - b / d) * sigma_j / |b_j|, 0 where d = 0),
 * T[k * ceil(n/64)][64]; scales from ttn_precond_features. */
ttn_status ttn_precond_targets(ttn_ctx* ctx, int32_t k, int64_t n, ttn_dtype storage, const void* y, const void* b,
                               const void* d, const double* scales, float* T);
/* Training pairs of the current local problems of a sweep at `node` (the
 * sweep's orthogonality centre): features of (b_j, diag(H_eff) - s_j) into
 * X[k * ceil(n/64)][128] and targets of the current local tensors (the
 * solution a MINRES step just left there) into T[k * ceil(n/64)][64];
 * scales double[k][2]. */
ttn_status ttn_sweep_harvest(ttn_ctx* ctx, ttn_sweep* sw, int32_t node, float* X, float* T, double* scales);

/* Algorithmic flop count of one heff_apply_block call for k states at node u
 * (minimum over pairwise contraction orders, dense operands at unpadded
 * shapes, per-state environments), and of one ttno_env_update per pair. */
ttn_status ttn_flops_heff(const ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_envs* envs,
                          int32_t node, int32_t k, double* flops);
ttn_status ttn_flops_env(const ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op, const ttn_block* bra,
                         const ttn_block* ket, int32_t node, int32_t toward, double* flops_per_pair);

#ifdef __cplusplus
}
#endif
#endif /* TTN_H */
