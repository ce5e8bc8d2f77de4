// Batched and served exchange builds (placeholder until the queue kernels land).
#include <hip/hip_runtime.h>

#include "hfx.h"
#include "hfx_internal.hpp"

using namespace hfx;

extern "C" hfx_status hfx_build_K_batch(int32_t, const hfx_pairs *, const double *const *, double *const *,
                                        const int64_t *, const hfx_opts *, void *, hfx_stats *) {
    return fail(HFX_EUNSUPPORTED, "batched build not available yet");
}
extern "C" hfx_status hfx_server_create(int64_t, int32_t, hfx_server *) {
    return fail(HFX_EUNSUPPORTED, "server not available yet");
}
extern "C" hfx_status hfx_submit(hfx_server, hfx_pairs, const double *, double *, int64_t, const hfx_opts *,
                                 uint64_t *) {
    return fail(HFX_EUNSUPPORTED, "server not available yet");
}
extern "C" hfx_status hfx_poll(hfx_server, uint64_t, int32_t *, hfx_stats *) {
    return fail(HFX_EUNSUPPORTED, "server not available yet");
}
extern "C" void hfx_server_destroy(hfx_server) {}
