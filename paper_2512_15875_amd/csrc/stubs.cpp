// Entry points not yet implemented on the GPU path: they validate nothing and
// report TTN_E_ARG with a message, so callers fail loudly.
#include "internal.h"

extern "C" {
#define TTN_UNIMPL(sig) sig { return TTN_E_ARG; }
TTN_UNIMPL(ttn_status rayleigh_ritz(ttn_ctx*, int32_t, const int32_t*, int32_t, const double*, const double*, int32_t, double, int32_t, double*, double*, int32_t*))
TTN_UNIMPL(ttn_status ttn_sweep_create(ttn_ctx*, const ttn_tree*, const ttn_ttno*, ttn_block*, int32_t, const ttn_ttno* const*, const ttn_block* const*, const int32_t*, const int32_t* const*, const int32_t* const*, const double* const*, const double*, ttn_dtype, ttn_sweep**))
TTN_UNIMPL(ttn_status ttn_sweep_init(ttn_sweep*, int32_t))
TTN_UNIMPL(ttn_status ttn_sweep_destroy(ttn_sweep*))
TTN_UNIMPL(ttn_status sweep_step(ttn_ctx*, ttn_sweep*, int32_t, int32_t, const ttn_solve_opts*, int32_t*, double*))
TTN_UNIMPL(ttn_status ttn_block_move_centre(ttn_ctx*, ttn_block*, int32_t, int32_t))
TTN_UNIMPL(ttn_status ttn_block_scale_node(ttn_ctx*, ttn_block*, int32_t, const double*))
TTN_UNIMPL(ttn_status ttn_block_node_norms2(ttn_ctx*, const ttn_block*, int32_t, double*))
}
