// heff_apply_block for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation):
// the contraction intermediates of the H_eff product live in a file-scope
// device array instead of the context workspace.  The kernels are the same as
// heff_apply_block's; only the workspace differs.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;  // 256 MiB per device, held until the process ends
constexpr int kMaxDevices = 64;

// One copy per device.  In host code this name is only a stand-in for the
// device symbol: host code uses the address looked up below, never the name.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

}  // namespace

namespace ttn {

// Called by ttn_ctx_create with `device` current: the address of this
// device's copy of `scratch`, looked up once per device.
bool noalloc_scratch_setup(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return false;
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return true;
}

}  // namespace ttn

extern "C" ttn_status heff_apply_block_noalloc(ttn_ctx* ctx, const ttn_tree* t, const ttn_ttno* op,
                                               const ttn_envs* envs, int32_t node, int32_t k, const int32_t* pair_ids,
                                               const int32_t* x_ids, const double* shift, const double* alpha,
                                               const void* X, int32_t x_rows, void* Y, uint32_t flags,
                                               ttn_dtype compute) {
  if (!ctx) return ttn::api_fail(nullptr, TTN_E_ARG, "null context");
  if (!ctx->scratch)
    return ttn::api_fail(ctx, TTN_E_DEVICE, "the static scratch array could not be located on this device");
  // the same launches as heff_apply_block, with the static array as workspace
  // (its previous contents are never read: every intermediate is written
  // before it is used)
  void* const ws = ctx->ws;
  const size_t wb = ctx->ws_bytes;
  ctx->ws = ctx->scratch;
  ctx->ws_bytes = kScratchBytes;
  ttn_status r = ttn::heff_apply_rows(ctx, t, op, envs, node, k, pair_ids, x_ids, nullptr, k, shift, alpha, X,
                                      x_rows, Y, flags, compute);
  ctx->ws = ws;
  ctx->ws_bytes = wb;
  if (r == TTN_E_WORKSPACE)
    return ttn::api_fail(ctx, TTN_E_WORKSPACE,
                         "one state's contraction intermediates exceed the 256 MiB static scratch; use heff_apply_block");
  return r;
}
