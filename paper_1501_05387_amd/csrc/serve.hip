// serve.hip -- asynchronous query serving (submit / poll / cancel).
#include "engine.h"

namespace gfr {
struct Server {};

void serve_shutdown(Ctx &c)
{
    delete c.server;
    c.server = nullptr;
}
}  // namespace gfr

using namespace gfr;

extern "C" {

gfr_status gfr_submit_queries(gfr_ctx *ctx, const gfr_query *q, int32_t count, gfr_ticket *tickets_out)
{
    (void)q; (void)count; (void)tickets_out;
    if (!ctx) return GFR_E_INVALID;
    ((Ctx *)ctx)->err = "serving not available in this build";
    return GFR_E_INVALID;
}

gfr_status gfr_poll(gfr_ctx *ctx, gfr_ticket *done, gfr_status *status, int32_t cap, int32_t *ndone,
                    int32_t timeout_us)
{
    (void)done; (void)status; (void)cap; (void)timeout_us;
    if (!ctx) return GFR_E_INVALID;
    if (ndone) *ndone = 0;
    return GFR_OK;
}

gfr_status gfr_cancel(gfr_ctx *ctx, gfr_ticket t)
{
    (void)t;
    if (!ctx) return GFR_E_INVALID;
    return GFR_E_NOT_FOUND;
}

}  // extern "C"
