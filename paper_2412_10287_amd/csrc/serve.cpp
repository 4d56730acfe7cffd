// Served path: rpq_submit / rpq_poll.
#include "api_internal.h"

using namespace rpq;

void rpq::serve_shutdown(rpq_graph *) {}
bool rpq::serve_pending(rpq_graph *) { return false; }
void rpq::batch_free(rpq_graph *) {}

rpq_status rpq_multi_source(rpq_graph *g, const rpq_nfa *n, const int32_t *sources, int32_t n_sources,
                            uint64_t *out_bitmaps, uint32_t flags, rpq_stats *stats) {
    (void)g; (void)n; (void)sources; (void)n_sources; (void)out_bitmaps; (void)flags; (void)stats;
    return fail(RPQ_EINVAL, "rpq_multi_source: not built yet");
}

rpq_status rpq_submit(rpq_graph *g, const rpq_nfa *n, int32_t source, rpq_ticket *out) {
    (void)g; (void)n; (void)source; (void)out;
    return fail(RPQ_EINVAL, "rpq_submit: not built yet");
}

rpq_status rpq_poll(rpq_graph *g, rpq_ticket t, uint64_t *out_bitmap, rpq_stats *stats, int64_t timeout_us) {
    (void)g; (void)t; (void)out_bitmap; (void)stats; (void)timeout_us;
    return fail(RPQ_EINVAL, "rpq_poll: not built yet");
}
