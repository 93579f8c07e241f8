// Serving loop of libompd (continuous batching); see include/ompd.h.
#include <hip/hip_runtime.h>

#include "ompd_internal.h"

void ompd_serving_shutdown(ompd_ctx*) {}

extern "C" int ompd_submit(ompd_ctx*, const ompd_cfg*, ompd_result*, uint32_t, ompd_ticket*)
{
    return ompd_fail(OMPD_E_INVAL, "serving not built yet");
}
extern "C" int ompd_poll(ompd_ctx*, ompd_ticket, int*) { return OMPD_E_UNKNOWN_TICKET; }
extern "C" int ompd_wait(ompd_ctx*, ompd_ticket, int64_t, int*) { return OMPD_E_UNKNOWN_TICKET; }
extern "C" int ompd_serving_stats(ompd_ctx*, int64_t*, int64_t*, int64_t*, int64_t*) { return OMPD_OK; }
