// Autotuner: times candidate settings of the plain or the stacked path on a
// sample of queries and keeps the fastest on the graph handle.
//
// The knobs are the ones the hardware makes worth measuring rather than
// guessing: the number of workgroups of the persistent single-query launch
// (fewer workgroups make each grid barrier cheaper, more of them spread large
// levels wider) and the push -> pull / pull -> push thresholds of the
// direction switch. The paper's own hybrid switches between its two
// formulations at a fixed constant (Sec. 5.1); on the GPU the best switch
// point depends on the graph's degree skew and the queries' label mix, so it
// is measured.
#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "api_internal.h"

using namespace rpq;

// the Python binding mirrors this layout field by field
static_assert(offsetof(rpq_tuning, handoff_edges) == 48 && sizeof(rpq_tuning) == 56, "rpq_tuning layout");

namespace {

struct Setting {
    int32_t grid;
    double alpha, beta;
    int64_t handoff;  // stacked: phase-kernel hand-off threshold
};

rpq_status time_plain(rpq_graph *g, const rpq_nfa *const *nfas, const int32_t *src, int32_t n, double *ms) {
    *ms = 0.0;
    for (int32_t i = 0; i < n; i++) {
        rpq_stats st{};
        const rpq_status r = run_single(g, nfas[i], src[i], g->dev_out, RPQ_OUT_DEVICE, &st);
        if (r != RPQ_OK) return r;
        *ms += st.device_ms;
    }
    return RPQ_OK;
}

rpq_status time_stacked(rpq_graph *g, const rpq_nfa *nfa, const int32_t *src, int32_t n, uint64_t *dout,
                        double *ms) {
    rpq_stats st{};
    const rpq_status r = rpq_multi_source(g, nfa, src, n, dout, RPQ_OUT_DEVICE, &st);
    *ms = st.device_ms;
    return r;
}

}  // namespace

rpq_status rpq_autotune(rpq_graph *g, int32_t path, const rpq_nfa *const *nfas, const int32_t *sources,
                        int32_t n_queries, rpq_tuning *out) {
    if (!g || !nfas || !sources || !out) return fail(RPQ_EINVAL, "rpq_autotune: NULL argument");
    if (path != RPQ_TUNE_PLAIN && path != RPQ_TUNE_STACKED) return fail(RPQ_EINVAL, "rpq_autotune: unknown path %d", path);
    if (n_queries < 1) return fail(RPQ_EINVAL, "rpq_autotune: n_queries < 1");
    const int32_t nn = path == RPQ_TUNE_PLAIN ? n_queries : 1;
    for (int32_t i = 0; i < nn; i++)
        if (!nfas[i]) return fail(RPQ_EINVAL, "rpq_autotune: NULL automaton %d", i);
    for (int32_t i = 0; i < n_queries; i++)
        if (sources[i] < 0 || sources[i] >= g->V)
            return fail(RPQ_EINVAL, "rpq_autotune: source %d outside [0, %d)", sources[i], g->V);
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    if (hipSetDevice(g->device) != hipSuccess) return fail(RPQ_EDEVICE, "rpq_autotune: hipSetDevice failed");
    // candidates
    std::vector<Setting> cand;
    const double alphas[] = {0.0, 1.0, 2.0, 4.0, 8.0, 16.0, 64.0};
    const double betas[] = {4.0, 24.0, 128.0};
    int32_t grids[4] = {0, 0, 0, 0};
    int32_t ng = 1;
    if (path == RPQ_TUNE_PLAIN) {
        const int32_t full = g->pgrid[1];
        grids[0] = 0;  // one workgroup per CU
        for (int32_t d : {2, 4, 8})
            if (full / d >= 16) grids[ng++] = full / d;
    }
    // saved settings (restored on failure), and the time with them
    const int32_t grid0 = g->plain_grid;
    const double a0 = path == RPQ_TUNE_PLAIN ? g->pull_alpha : g->stack_alpha;
    const double b0 = path == RPQ_TUNE_PLAIN ? g->pull_beta : g->stack_beta;
    const int64_t h0 = g->stack_handoff;
    for (int32_t gi = 0; gi < ng; gi++)
        for (double a : alphas) {
            if (a == 0.0) {
                cand.push_back({grids[gi], 0.0, 24.0, h0});
                continue;
            }
            for (double b : betas) cand.push_back({grids[gi], a, b, h0});
        }
    auto apply = [&](const Setting &s) {
        if (path == RPQ_TUNE_PLAIN) {
            g->plain_grid = s.grid;
            g->pull_alpha = s.alpha;
            g->pull_beta = s.beta;
        } else {
            g->stack_alpha = s.alpha;
            g->stack_beta = s.beta;
            g->stack_handoff = s.handoff;
        }
    };
    uint64_t *dout = nullptr;
    if (path == RPQ_TUNE_STACKED) {
        const size_t bytes = 8 * static_cast<size_t>(n_queries) * static_cast<size_t>(g->nwords);
        if (hipMalloc(reinterpret_cast<void **>(&dout), bytes) != hipSuccess)
            return fail(RPQ_ENOMEM, "rpq_autotune: hipMalloc of %zu bytes", bytes);
    }
    auto measure = [&](double *ms) -> rpq_status {
        return path == RPQ_TUNE_PLAIN ? time_plain(g, nfas, sources, n_queries, ms)
                                      : time_stacked(g, nfas[0], sources, n_queries, dout, ms);
    };
    rpq_status st;
    double def_ms = 0.0, best_ms = 0.0;
    Setting best{grid0, a0, b0, h0};
    // warm-up with the saved settings, then their time
    if ((st = measure(&def_ms)) == RPQ_OK) st = measure(&def_ms);
    best_ms = def_ms;
    auto try_setting = [&](const Setting &c) {
        apply(c);
        double ms = 0.0;
        st = measure(&ms);
        if (st == RPQ_OK && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    };
    for (size_t k = 0; st == RPQ_OK && k < cand.size(); k++) try_setting(cand[k]);
    size_t ncand = cand.size();
    // stacked, second stage: the hand-off threshold under the best
    // direction thresholds (the two interact little: pull levels never
    // leave the persistent kernel)
    if (path == RPQ_TUNE_STACKED) {
        const Setting base = best;  // the first stage's choice (threshold h0)
        for (int64_t h : {int64_t{0}, int64_t{1} << 20, int64_t{1} << 22, int64_t{1} << 24}) {
            if (st != RPQ_OK || h == base.handoff) continue;
            Setting c = base;
            c.handoff = h;
            try_setting(c);
            ncand++;
        }
    }
    if (dout) (void)hipFree(dout);
    apply(st == RPQ_OK ? best : Setting{grid0, a0, b0, h0});
    if (st != RPQ_OK) return st;
    out->grid = best.grid;
    out->alpha = static_cast<int64_t>(best.alpha);
    out->beta = static_cast<int64_t>(best.beta);
    out->best_ms = best_ms;
    out->default_ms = def_ms;
    out->candidates = static_cast<int32_t>(ncand);
    out->handoff_edges = path == RPQ_TUNE_STACKED ? best.handoff : 0;
    return RPQ_OK;
}
