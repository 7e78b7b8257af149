// Serving loop (continuous batching over the resident index).
#include "runtime.h"

using namespace lnbnn;

namespace lnbnn {
struct Server {};
void server_stop(lnbnn_index *) {}
bool server_pending(lnbnn_index *) { return false; }
}  // namespace lnbnn

extern "C" int lnbnn_submit(lnbnn_index *ix, const void *, int, int64_t, int32_t, int, uint64_t *)
{
    if (!ix) return set_err(LNBNN_EINVAL, "NULL index");
    return set_err(LNBNN_EINVAL, "serving is not built yet");
}

extern "C" int lnbnn_poll(lnbnn_index *ix, uint64_t, int32_t *, void *, lnbnn_req_stats *)
{
    if (!ix) return set_err(LNBNN_EINVAL, "NULL index");
    return set_err(LNBNN_ENOENT, "unknown ticket");
}

extern "C" int lnbnn_serve_config(lnbnn_index *ix, int64_t, int32_t)
{
    if (!ix) return set_err(LNBNN_EINVAL, "NULL index");
    return LNBNN_OK;
}
