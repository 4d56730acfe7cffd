// C-ABI entry points of librpq (declared in include/rpq.h) and the host
// runtime behind them: graph upload, per-query NFA tables, the single-query
// executor (one persistent launch, or a host-driven level loop).
#include "api_internal.h"
#include "trace.h"

#include <stdarg.h>
#include <stdio.h>
#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>

using namespace rpq;

// ------------------------------------------------------------------ errors
static thread_local char g_err[512] = "";

const char *rpq_last_error(void) { return g_err; }

rpq_status rpq::fail(rpq_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

// Persistent grids wait for all of their workgroups at grid barriers, so all
// of them must be resident at once; two grids in flight on one device that
// together do not fit could each hold part of the GPU and wait (up to the
// barrier timeout) for workgroups that cannot start. Every persistent launch
// of this process therefore takes its workgroups from a per-device budget of
// two per compute unit, from the launch until its stream has drained it, and
// waits in arrival order while the budget is short. A workgroup of a kernel
// that fits at least twice per compute unit (512 threads, so at most 128
// VGPRs and 80 KB of LDS) costs one unit: any two such workgroups fit on one
// compute unit together. Other kernels cost two.
namespace {
struct Budget {
    std::mutex mu;
    std::condition_variable cv;
    int64_t total = -1;  // units, set at first use
    int64_t free = 0;
    uint64_t next = 0, serving = 0;  // arrival tickets
};
Budget &budget_of(int device) {
    static Budget b[64];
    return b[static_cast<unsigned>(device) & 63u];
}
}  // namespace

rpq_status rpq::PersistentHold::acquire(int device, int grid, int blocks_per_cu) {
    release();
    Budget &b = budget_of(device);
    std::unique_lock<std::mutex> lk(b.mu);
    if (b.total < 0) {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu < 1)
            return fail(RPQ_EDEVICE, "hipDeviceGetAttribute(multiprocessor count) failed");
        b.total = 2 * static_cast<int64_t>(ncu);
        b.free = b.total;
    }
    int64_t units = static_cast<int64_t>(grid) * (blocks_per_cu >= 2 ? 1 : 2);
    units = std::min(units, b.total);
    const uint64_t me = b.next++;
    b.cv.wait(lk, [&] { return b.serving == me && b.free >= units; });
    b.serving++;
    b.free -= units;
    b.cv.notify_all();  // the next arrival may fit as well
    device_ = device;
    units_ = units;
    return RPQ_OK;
}

void rpq::PersistentHold::release() {
    if (device_ < 0) return;
    Budget &b = budget_of(device_);
    {
        std::lock_guard<std::mutex> lk(b.mu);
        b.free += units_;
    }
    b.cv.notify_all();
    device_ = -1;
    units_ = 0;
}

rpq_status rpq::hip_fail(hipError_t e, const char *what) {
    return fail(RPQ_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

void rpq::stats_reset(rpq_stats *st) {
    rpq_stats in = *st;
    *st = rpq_stats{};
    st->level_counts = in.level_counts;
    st->level_cap = in.level_cap;
    st->level_us = in.level_us;
    st->level_frontier = in.level_frontier;
    st->level_edges = in.level_edges;
    st->level_select_us = in.level_select_us;
}

int64_t rpq::stats_levels(rpq_stats *st, const uint64_t *lvl, uint32_t nrec, uint32_t levels) {
    int64_t visited = 0;
    const uint32_t nl = std::min(nrec, levels);
    for (uint32_t i = 0; i < nl; i++) visited += static_cast<int64_t>(lvl[static_cast<size_t>(i) * LVL_STRIDE]);
    if (!st || st->level_cap <= 0) return visited;
    for (int32_t i = 0; i < st->level_cap; i++) {
        const bool have = static_cast<uint32_t>(i) < nl;
        const uint64_t *r = lvl + static_cast<size_t>(i) * LVL_STRIDE;
        if (st->level_counts) st->level_counts[i] = have ? static_cast<int64_t>(r[0]) : 0;
        if (st->level_frontier) st->level_frontier[i] = have ? static_cast<int64_t>(r[1]) : 0;
        if (st->level_edges) st->level_edges[i] = have ? static_cast<int64_t>(r[2] & 0xffffffffull) : 0;
        if (st->level_select_us)
            st->level_select_us[i] = have && r[4] > r[3] ? static_cast<double>(r[4] - r[3]) * 0.01 : 0.0;
        if (st->level_us) {
            // the device wall clock runs at 100 MHz
            const bool end = have && static_cast<uint32_t>(i) + 1 < nrec;
            st->level_us[i] = end ? static_cast<double>(r[LVL_STRIDE + 3] - r[3]) * 0.01 : 0.0;
        }
    }
    return visited;
}

int64_t rpq_bitmap_words(int32_t num_vertices) {
    return num_vertices > 0 ? (static_cast<int64_t>(num_vertices) + 63) / 64 : 0;
}

// ------------------------------------------------------------------ NFA
rpq_status rpq_nfa_load(int32_t num_states, int32_t num_labels, const int64_t *sym_ptr,
                        const int32_t *from, const int32_t *to, const int32_t *start, int32_t n_start,
                        const int32_t *final_states, int32_t n_final, rpq_nfa **out) {
    if (!out) return fail(RPQ_EINVAL, "rpq_nfa_load: out is NULL");
    *out = nullptr;
    if (num_states < 1 || num_states > MAX_STATES)
        return fail(RPQ_EINVAL, "rpq_nfa_load: num_states %d outside [1, %d]", num_states, MAX_STATES);
    if (num_labels < 0) return fail(RPQ_EINVAL, "rpq_nfa_load: num_labels < 0");
    if (!sym_ptr) return fail(RPQ_EINVAL, "rpq_nfa_load: sym_ptr is NULL");
    if (n_start < 0 || n_final < 0) return fail(RPQ_EINVAL, "rpq_nfa_load: negative count");
    if ((n_start && !start) || (n_final && !final_states))
        return fail(RPQ_EINVAL, "rpq_nfa_load: NULL start/final array");
    const int64_t nsym = 2 * static_cast<int64_t>(num_labels);
    if (sym_ptr[0] != 0) return fail(RPQ_EINVAL, "rpq_nfa_load: sym_ptr[0] != 0");
    for (int64_t s = 0; s < nsym; s++)
        if (sym_ptr[s + 1] < sym_ptr[s]) return fail(RPQ_EINVAL, "rpq_nfa_load: sym_ptr decreases at %lld", (long long)s);
    const int64_t nt = sym_ptr[nsym];
    if (nt && (!from || !to)) return fail(RPQ_EINVAL, "rpq_nfa_load: NULL transition arrays");
    for (int64_t i = 0; i < nt; i++)
        if (from[i] < 0 || from[i] >= num_states || to[i] < 0 || to[i] >= num_states)
            return fail(RPQ_EINVAL, "rpq_nfa_load: transition %lld has a state out of range", (long long)i);
    uint32_t sm = 0, fm = 0;
    for (int32_t i = 0; i < n_start; i++) {
        if (start[i] < 0 || start[i] >= num_states) return fail(RPQ_EINVAL, "rpq_nfa_load: start state out of range");
        sm |= 1u << start[i];
    }
    for (int32_t i = 0; i < n_final; i++) {
        if (final_states[i] < 0 || final_states[i] >= num_states)
            return fail(RPQ_EINVAL, "rpq_nfa_load: final state out of range");
        fm |= 1u << final_states[i];
    }
    rpq_nfa *n = new (std::nothrow) rpq_nfa;
    if (!n) return fail(RPQ_ENOMEM, "rpq_nfa_load: out of host memory");
    n->Q = num_states;
    n->NL = num_labels;
    n->smask = sm;
    n->fmask = fm;
    static std::atomic<uint64_t> serial{1};
    n->serial = serial.fetch_add(1);
    for (int64_t s = 0; s < nsym; s++)
        for (int64_t i = sym_ptr[s]; i < sym_ptr[s + 1]; i++)
            n->trans.push_back({static_cast<int32_t>(s), from[i], to[i]});
    *out = n;
    return RPQ_OK;
}

rpq_status rpq_nfa_free(rpq_nfa *n) {
    delete n;
    return RPQ_OK;
}

// Builds the query-constant block (QHeader, succ, pred, label->symbol maps)
// for NFA n on graph g into dst (cap bytes), with no heap allocation; returns
// its size in bytes, or 0 when n uses more than MAX_SYMS symbols (*nsym_out
// says how many) or the block would exceed cap.
size_t rpq::build_qconst_into(const rpq_graph *g, const rpq_nfa *n, uint32_t force, uint32_t counters, uint8_t *dst,
                              size_t cap, int32_t *nsym_out) {
    const int32_t L = g->L;
    // used symbols: label within the graph, with edges, with transitions; in
    // order of first transition
    int32_t used[MAX_SYMS];
    int32_t ns = 0;
    bool over = false;
    auto index_of = [&](int32_t sym) {
        for (int32_t u = 0; u < ns; u++)
            if (used[u] == sym) return u;
        return -1;
    };
    int32_t total = 0;
    for (const auto &t : n->trans) {
        const int32_t lab = t.sym >= n->NL ? t.sym - n->NL : t.sym;
        if (lab >= L || g->label_edges[lab] == 0) continue;
        if (index_of(t.sym) >= 0) continue;
        if (ns < MAX_SYMS) used[ns++] = t.sym;
        else over = true;
        total++;
    }
    if (over) {
        // count the distinct used symbols beyond the table for the message
        total = ns;
        for (size_t i = 0; i < n->trans.size(); i++) {
            const Trans &t = n->trans[i];
            const int32_t lab = t.sym >= n->NL ? t.sym - n->NL : t.sym;
            if (lab >= L || g->label_edges[lab] == 0 || index_of(t.sym) >= 0) continue;
            bool seen = false;
            for (size_t k = 0; k < i && !seen; k++) seen = n->trans[k].sym == t.sym;
            if (!seen) total++;
        }
        *nsym_out = total;
        return 0;
    }
    *nsym_out = ns;
    const size_t sz = qconst_bytes(static_cast<size_t>(ns));
    if (sz > cap) return 0;
    memset(dst, 0, sz);
    const QOffsets o = qconst_offsets(static_cast<size_t>(ns));
    QHeader *h = reinterpret_cast<QHeader *>(dst);
    uint64_t *symmask = reinterpret_cast<uint64_t *>(dst + o.symmask);
    uint32_t *succ = reinterpret_cast<uint32_t *>(dst + o.succ);
    uint32_t *pred = reinterpret_cast<uint32_t *>(dst + o.pred);
    uint64_t *push_w = reinterpret_cast<uint64_t *>(dst + o.push_w);
    uint64_t *pull_w = reinterpret_cast<uint64_t *>(dst + o.pull_w);
    uint32_t *push_r = reinterpret_cast<uint32_t *>(dst + o.push_r);
    uint32_t *pull_r = reinterpret_cast<uint32_t *>(dst + o.pull_r);
    uint32_t *pull_n = reinterpret_cast<uint32_t *>(dst + o.pull_n);
    h->Q = n->Q;
    h->nsym = ns;
    h->smask = n->smask;
    h->fmask = n->fmask;
    h->alpha = static_cast<float>(g->pull_alpha);
    h->beta = static_cast<float>(g->pull_beta);
    h->force = force;
    h->counters = counters;
    uint64_t erel = 0;
    for (int32_t u = 0; u < ns; u++) {
        const int32_t s = used[u];
        const bool inv = s >= n->NL;
        const int32_t lab = inv ? s - n->NL : s;
        // a forward symbol follows G^a (OUT rows) when pushing and (G^a)^T when
        // pulling; an inverse symbol the other way round (G^{a^-} = (G^a)^T)
        const int dpush = inv ? IN : OUT, dpull = inv ? OUT : IN;
        push_w[u] = (static_cast<uint64_t>(dpush) * L + lab) * static_cast<uint64_t>(g->nwords);
        pull_w[u] = (static_cast<uint64_t>(dpull) * L + lab) * static_cast<uint64_t>(g->nwords);
        push_r[u] = static_cast<uint32_t>(g->rbase[static_cast<size_t>(dpush) * L + lab]);
        pull_r[u] = static_cast<uint32_t>(g->rbase[static_cast<size_t>(dpull) * L + lab]);
        pull_n[u] = static_cast<uint32_t>(g->label_rows[static_cast<size_t>(dpull)][lab]);
        erel += static_cast<uint64_t>(g->label_edges[lab]);
    }
    for (const auto &t : n->trans) {
        const int32_t u = index_of(t.sym);
        if (u < 0) continue;
        succ[u * MAX_STATES + t.from] |= 1u << t.to;
        pred[u * MAX_STATES + t.to] |= 1u << t.from;
        symmask[t.from * SYM_WORDS + u / 64] |= 1ull << (u % 64);
        h->inmask |= 1u << t.to;
        h->succ_any[t.from] |= 1u << t.to;
    }
    h->e_rel = erel;
    return sz;
}

// The same into a vector sized to the block.
size_t rpq::build_qconst(const rpq_graph *g, const rpq_nfa *n, uint32_t force, uint32_t counters,
                         std::vector<uint8_t> &buf, int32_t *nsym_out) {
    buf.resize(qconst_bytes(MAX_SYMS));
    const size_t sz = build_qconst_into(g, n, force, counters, buf.data(), buf.size(), nsym_out);
    buf.resize(sz);
    return sz;
}

// Device addresses of the tables inside a query-constant block at `base`.
QueryView rpq::query_view(uint8_t *base, int32_t nsym) { return qconst_view(base, static_cast<size_t>(nsym)); }

// ------------------------------------------------------------------ graph
static rpq_status dev_alloc(rpq_graph *g, void **p, size_t bytes, const char *what) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 64);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(RPQ_ENOMEM, "hipMalloc(%s, %zu bytes): %s", what, bytes, hipGetErrorString(e));
    }
    g->allocs.push_back(*p);
    g->device_bytes += static_cast<int64_t>(bytes);
    return RPQ_OK;
}

template <typename T>
static rpq_status upload(rpq_graph *g, T **dst, const std::vector<T> &src, const char *what) {
    rpq_status st = dev_alloc(g, reinterpret_cast<void **>(dst), src.size() * sizeof(T), what);
    if (st != RPQ_OK) return st;
    if (!src.empty()) HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return RPQ_OK;
}

static void destroy(rpq_graph *g) {
    if (!g) return;
    serve_shutdown(g);
    for (hipGraphExec_t &ex : g->lgraph)
        if (ex) (void)hipGraphExecDestroy(ex);
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    for (hipEvent_t e : g->ev)
        if (e) (void)hipEventDestroy(e);
    if (g->pinned) (void)hipHostFree(g->pinned);
    if (g->hstat) (void)hipHostFree(g->hstat);
    if (g->pin_srcset) (void)hipHostFree(g->pin_srcset);
    for (void *p : g->allocs) (void)hipFree(p);
    batch_free(g);
    delete g;
}

rpq_status rpq_graph_load(int32_t V, int32_t L, const int64_t *label_ptr, const int32_t *src,
                          const int32_t *dst, rpq_graph **out) {
    TraceRange tr_("rpq_graph_load");
    if (!out) return fail(RPQ_EINVAL, "rpq_graph_load: out is NULL");
    *out = nullptr;
    if (V < 1) return fail(RPQ_EINVAL, "rpq_graph_load: num_vertices < 1");
    if (L < 1) return fail(RPQ_EINVAL, "rpq_graph_load: num_labels < 1");
    if (!label_ptr) return fail(RPQ_EINVAL, "rpq_graph_load: label_ptr is NULL");
    if (label_ptr[0] != 0) return fail(RPQ_EINVAL, "rpq_graph_load: label_ptr[0] != 0");
    for (int32_t l = 0; l < L; l++)
        if (label_ptr[l + 1] < label_ptr[l]) return fail(RPQ_EINVAL, "rpq_graph_load: label_ptr decreases at %d", l);
    const int64_t E = label_ptr[L];
    if (E > 0 && (!src || !dst)) return fail(RPQ_EINVAL, "rpq_graph_load: NULL edge arrays");
    if (E > MAX_EDGES) return fail(RPQ_EINVAL, "rpq_graph_load: %lld edges exceed the limit %lld",
                                   (long long)E, (long long)MAX_EDGES);
    for (int64_t i = 0; i < E; i++)
        if (src[i] < 0 || src[i] >= V || dst[i] < 0 || dst[i] >= V)
            return fail(RPQ_EINVAL, "rpq_graph_load: edge %lld has a vertex id out of range", (long long)i);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(RPQ_EDEVICE, "rpq_graph_load: no HIP device is available");

    rpq_graph *g = new (std::nothrow) rpq_graph;
    if (!g) return fail(RPQ_ENOMEM, "rpq_graph_load: out of host memory");
    g->V = V;
    g->L = L;
    rpq_status st = graph_upload(g, label_ptr, src, dst);
    if (st != RPQ_OK) {
        destroy(g);
        return st;
    }
    *out = g;
    return RPQ_OK;
}

rpq_status rpq::graph_upload(rpq_graph *g, const int64_t *label_ptr, const int32_t *src, const int32_t *dst) {
    const int32_t V = g->V, L = g->L;
    HIP_TRY(hipGetDevice(&g->device));
    rpq_status st;
    HostDir d[2];
    build_direction(V, src, dst, label_ptr, L, 0, d[OUT]);
    const int64_t E = d[OUT].E;
    build_direction(V, dst, src, label_ptr, L, static_cast<uint32_t>(E), d[IN]);
    g->E = E;
    g->label_edges = d[OUT].label_edges;
    g->label_rows[OUT] = d[OUT].label_rows;
    g->label_rows[IN] = d[IN].label_rows;
    g->nwords = rpq_bitmap_words(V);
    g->rows[OUT] = g->rows[IN] = 0;
    for (int32_t l = 0; l < L; l++) {
        g->rows[OUT] += d[OUT].label_rows[l];
        g->rows[IN] += d[IN].label_rows[l];
    }
    // one array per kind, OUT part first
    const uint64_t nrp_out = d[OUT].rowptr.size();
    g->rbase.assign(2 * static_cast<size_t>(L), 0);
    for (int32_t l = 0; l < L; l++) {
        g->rbase[l] = d[OUT].rbase[l];
        g->rbase[L + l] = nrp_out + d[IN].rbase[l];
    }
    uint32_t *col = nullptr, *rowptr = nullptr, *rowvert = nullptr;
    RankWordD *rankw = nullptr;
    const size_t nrank = static_cast<size_t>(L) * g->nwords;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&col), 2 * E * sizeof(uint32_t), "col")) != RPQ_OK) return st;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&rowptr),
                        (nrp_out + d[IN].rowptr.size()) * sizeof(uint32_t), "rowptr")) != RPQ_OK)
        return st;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&rowvert),
                        (nrp_out + d[IN].rowptr.size()) * sizeof(uint32_t), "rowvert")) != RPQ_OK)
        return st;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&rankw), 2 * nrank * sizeof(RankWordD), "rank")) != RPQ_OK)
        return st;
    static_assert(sizeof(RankWord) == sizeof(RankWordD), "rank word layout");
    for (int k = 0; k < 2; k++) {
        if (d[k].E)
            HIP_TRY(hipMemcpy(col + (k ? E : 0), d[k].col.data(), d[k].E * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(rowvert + (k ? nrp_out : 0), d[k].rowvert.data(), d[k].rowvert.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(rowptr + (k ? nrp_out : 0), d[k].rowptr.data(), d[k].rowptr.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(rankw + (k ? nrank : 0), d[k].rankw.data(), nrank * sizeof(RankWordD),
                          hipMemcpyHostToDevice));
        HostDir().col.swap(d[k].col);
    }
    g->gv.col = col;
    g->gv.rowptr = rowptr;
    g->gv.rowvert = rowvert;
    g->gv.rankw = rankw;
    g->gv.ncol = 2 * static_cast<uint64_t>(E);
    g->gv.nwords = g->nwords;
    g->gv.V = V;
    g->gv.L = L;
    return exec_alloc(g);
}

// The single-query executor's device state (sized for 4-byte state words),
// its pinned staging, stream and events: everything rpq_single_source needs
// besides the graph store.
rpq_status rpq::exec_alloc(rpq_graph *g) {
    const int32_t V = g->V;
    const int64_t E = g->E;
    rpq_status st;
    StateView &sv = g->sv;
    const size_t wbytes = 4 * static_cast<size_t>(V) + 256;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&sv.P), wbytes, "P")) != RPQ_OK) return st;
    for (int k = 0; k < 2; k++) {
        if ((st = dev_alloc(g, reinterpret_cast<void **>(&sv.M[k]), wbytes, "M")) != RPQ_OK) return st;
        if ((st = dev_alloc(g, reinterpret_cast<void **>(&sv.q[k]), 4 * static_cast<size_t>(V), "queue")) != RPQ_OK)
            return st;
    }
    // an item is one (vertex, label, direction) row: at most one per row and level
    sv.item_cap = static_cast<uint64_t>(g->rows[OUT] + g->rows[IN]) + 1;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&sv.it_ebase), 4 * sv.item_cap, "items")) != RPQ_OK) return st;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&sv.it_beg), 4 * sv.item_cap, "items")) != RPQ_OK) return st;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&sv.it_mask), 4 * sv.item_cap, "items")) != RPQ_OK) return st;
    sv.tile_cap = (2 * static_cast<uint64_t>(E)) / TILE + 2;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&sv.tile_first), 4 * sv.tile_cap, "tiles")) != RPQ_OK) return st;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&sv.rec), sizeof(LevelRec) * REC_RING, "rec")) != RPQ_OK) return st;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&sv.lvl), 8 * LVL_STRIDE * (LVL_COUNT_CAP + 1), "lvl")) !=
        RPQ_OK)
        return st;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&g->dev_out), 8 * g->nwords, "out")) != RPQ_OK) return st;
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&sv.cnt), 64, "cnt")) != RPQ_OK) return st;
    for (int k = 0; k < 2; k++)
        if ((st = dev_alloc(g, reinterpret_cast<void **>(&g->bars[k]), sizeof(GridBarrier), "barrier")) != RPQ_OK)
            return st;
    sv.bar = g->bars[0];
    sv.bar_next = g->bars[1];
    sv.status = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(sv.bar) + offsetof(GridBarrier, status));
    g->qconst_cap = qconst_bytes(MAX_SYMS) + 64;  // one query's constants at most
    if ((st = dev_alloc(g, reinterpret_cast<void **>(&g->qconst_dev), QARENA_BYTES, "qconst")) != RPQ_OK) return st;
    g->pinned_cap = g->qconst_cap + 4096 + 8 * LVL_STRIDE * (LVL_COUNT_CAP + 1);
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&g->pinned), g->pinned_cap, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&g->hstat), 64, hipHostMallocDefault));
    HIP_TRY(hipHostGetDevicePointer(reinterpret_cast<void **>(&g->hstat_dev), g->hstat, 0));
    memset(g->hstat, 0, 64);
    HIP_TRY(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
    g->own_stream = true;
    for (int k = 0; k < 4; k++) HIP_TRY(hipEventCreate(&g->ev[k]));
    // zero the query state once; every query leaves it zero again
    HIP_TRY(launch_fill(sv.P, wbytes / 4, 0, g->stream));
    HIP_TRY(launch_fill(sv.M[0], wbytes / 4, 0, g->stream));
    HIP_TRY(launch_fill(sv.M[1], wbytes / 4, 0, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    for (int W : {1, 2, 4}) g->pgrid[W] = persistent_grid(W);
    return RPQ_OK;
}

rpq_status rpq::exec_clone(const rpq_graph *g, rpq_graph **out) {
    *out = nullptr;
    HIP_TRY(hipSetDevice(g->device));
    rpq_graph *c = new (std::nothrow) rpq_graph;
    if (!c) return fail(RPQ_ENOMEM, "out of host memory");
    c->clone_of = g;
    c->V = g->V;
    c->L = g->L;
    c->E = g->E;
    c->device = g->device;
    c->gv = g->gv;
    c->label_edges = g->label_edges;
    for (int k = 0; k < 2; k++) {
        c->label_rows[k] = g->label_rows[k];
        c->rows[k] = g->rows[k];
    }
    c->rbase = g->rbase;
    c->nwords = g->nwords;
    exec_sync_options(c, g);
    const rpq_status st = exec_alloc(c);
    if (st != RPQ_OK) {
        destroy(c);
        return st;
    }
    *out = c;
    return RPQ_OK;
}

void rpq::exec_sync_options(rpq_graph *c, const rpq_graph *g) {
    c->pull_alpha = g->pull_alpha;
    c->pull_beta = g->pull_beta;
    c->plain_grid = g->plain_grid;
    c->grid_override = g->grid_override;
    c->coop_launch = g->coop_launch;
}

void rpq::exec_free(rpq_graph *c) { destroy(c); }

rpq_status rpq_graph_free(rpq_graph *g) {
    if (!g) return RPQ_OK;
    if (serve_pending(g)) return fail(RPQ_EAGAIN, "rpq_graph_free: tickets are still pending");
    destroy(g);
    return RPQ_OK;
}

rpq_status rpq_graph_info(const rpq_graph *g, const char *key, int64_t *value) {
    if (!g || !key || !value) return fail(RPQ_EINVAL, "rpq_graph_info: NULL argument");
    if (!strcmp(key, "num_vertices")) *value = g->V;
    else if (!strcmp(key, "num_labels")) *value = g->L;
    else if (!strcmp(key, "num_edges")) *value = g->E;
    else if (!strcmp(key, "device_bytes")) *value = g->device_bytes;
    else if (!strcmp(key, "rows_out")) *value = g->rows[OUT];
    else if (!strcmp(key, "rows_in")) *value = g->rows[IN];
    else if (!strcmp(key, "persistent_grid")) *value = g->pgrid[1];
    else if (!strcmp(key, "occupancy_blocks_per_cu")) *value = occupancy_blocks_per_cu(1);
    else if (!strcmp(key, "serve_slots")) *value = serve_slots(const_cast<rpq_graph *>(g));
    else if (!strcmp(key, "serve_lanes")) *value = serve_lane_count(const_cast<rpq_graph *>(g));
    else return fail(RPQ_ENOTFOUND, "rpq_graph_info: unknown key '%s'", key);
    return RPQ_OK;
}

rpq_status rpq_set_option(rpq_graph *g, const char *key, int64_t value) {
    if (!g || !key) return fail(RPQ_EINVAL, "rpq_set_option: NULL argument");
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    if (!strcmp(key, "stream")) {
        hipStream_t s = reinterpret_cast<hipStream_t>(static_cast<intptr_t>(value));
        g->user_stream = s;
    } else if (!strcmp(key, "pull_alpha")) {
        if (value < 0) return fail(RPQ_EINVAL, "rpq_set_option: pull_alpha < 0");
        g->pull_alpha = static_cast<double>(value);
    } else if (!strcmp(key, "pull_beta")) {
        if (value < 1) return fail(RPQ_EINVAL, "rpq_set_option: pull_beta < 1");
        g->pull_beta = static_cast<double>(value);
    } else if (!strcmp(key, "persistent_grid")) {
        if (value < 0) return fail(RPQ_EINVAL, "rpq_set_option: persistent_grid < 0");
        g->plain_grid = static_cast<int32_t>(std::min<int64_t>(value, 1 << 20));
    } else if (!strcmp(key, "stacked_alpha")) {
        if (value < 0) return fail(RPQ_EINVAL, "rpq_set_option: stacked_alpha < 0");
        g->stack_alpha = static_cast<double>(value);
    } else if (!strcmp(key, "stacked_beta")) {
        if (value < 1) return fail(RPQ_EINVAL, "rpq_set_option: stacked_beta < 1");
        g->stack_beta = static_cast<double>(value);
    } else if (!strcmp(key, "stacked_handoff_edges")) {
        if (value < 0 || value > (int64_t(1) << 40))
            return fail(RPQ_EINVAL, "rpq_set_option: stacked_handoff_edges outside [0, 2^40]");
        g->stack_handoff = value;
    } else if (!strcmp(key, "max_batch")) {
        if (value < 1 || value > MAX_BATCH) return fail(RPQ_EINVAL, "rpq_set_option: max_batch outside [1, %d]", MAX_BATCH);
        g->max_batch = static_cast<int32_t>(value);
    } else if (!strcmp(key, "mem_budget")) {
        if (value < 0) return fail(RPQ_EINVAL, "rpq_set_option: mem_budget < 0");
        g->mem_budget = value;
    } else if (!strcmp(key, "max_slots")) {
        if (value < 1 || value > MAX_SLOTS) return fail(RPQ_EINVAL, "rpq_set_option: max_slots outside [1, %d]", MAX_SLOTS);
        g->max_slots = static_cast<int32_t>(value);
    } else if (!strcmp(key, "large_query_pairs")) {
        if (value < 0) return fail(RPQ_EINVAL, "rpq_set_option: large_query_pairs < 0");
        g->large_pairs = value;
    } else if (!strcmp(key, "large_query_slots")) {
        if (value < 0 || value > MAX_SLOTS)
            return fail(RPQ_EINVAL, "rpq_set_option: large_query_slots outside [0, %d]", MAX_SLOTS);
        g->large_slots = static_cast<int32_t>(value);
    } else if (!strcmp(key, "rare_end_max")) {
        if (value < 0 || value > MAX_BATCH) return fail(RPQ_EINVAL, "rpq_set_option: rare_end_max outside [0, %d]", MAX_BATCH);
        g->rare_end_max = value;
    } else if (!strcmp(key, "serve_stack_min")) {
        if (value < 0 || value > MAX_BATCH)
            return fail(RPQ_EINVAL, "rpq_set_option: serve_stack_min outside [0, %d]", MAX_BATCH);
        g->serve_stack_min = static_cast<int32_t>(value);
    } else if (!strcmp(key, "serve_group_wait_us")) {
        if (value < 0 || value > 1000000)
            return fail(RPQ_EINVAL, "rpq_set_option: serve_group_wait_us outside [0, 10^6]");
        g->serve_group_wait_us = value;
    } else if (!strcmp(key, "serve_promote_pairs")) {
        if (value < 0) return fail(RPQ_EINVAL, "rpq_set_option: serve_promote_pairs < 0");
        g->serve_promote_pairs = value;
    } else if (!strcmp(key, "serve_lanes")) {
        if (value < 0 || value > MAX_LANES) return fail(RPQ_EINVAL, "rpq_set_option: serve_lanes outside [0, %d]", MAX_LANES);
        g->serve_lanes = static_cast<int32_t>(value);
    } else if (!strcmp(key, "cooperative_launch")) {
        if (value != 0 && value != 1) return fail(RPQ_EINVAL, "rpq_set_option: cooperative_launch must be 0 or 1");
        g->coop_launch = value != 0;
    } else if (!strcmp(key, "grid")) {
        if (value < 0) return fail(RPQ_EINVAL, "rpq_set_option: grid < 0");
        g->grid_override = static_cast<int32_t>(value);
    } else {
        return fail(RPQ_ENOTFOUND, "rpq_set_option: unknown key '%s'", key);
    }
    return RPQ_OK;
}

rpq_status rpq_get_option(const rpq_graph *g, const char *key, int64_t *value) {
    if (!g || !key || !value) return fail(RPQ_EINVAL, "rpq_get_option: NULL argument");
    if (!strcmp(key, "stream")) *value = static_cast<int64_t>(reinterpret_cast<intptr_t>(g->user_stream));
    else if (!strcmp(key, "pull_alpha")) *value = static_cast<int64_t>(g->pull_alpha);
    else if (!strcmp(key, "pull_beta")) *value = static_cast<int64_t>(g->pull_beta);
    else if (!strcmp(key, "persistent_grid")) *value = g->plain_grid;
    else if (!strcmp(key, "stacked_alpha")) *value = static_cast<int64_t>(g->stack_alpha);
    else if (!strcmp(key, "stacked_beta")) *value = static_cast<int64_t>(g->stack_beta);
    else if (!strcmp(key, "stacked_handoff_edges")) *value = g->stack_handoff;
    else if (!strcmp(key, "max_batch")) *value = g->max_batch;
    else if (!strcmp(key, "mem_budget")) *value = g->mem_budget;
    else if (!strcmp(key, "max_slots")) *value = g->max_slots;
    else if (!strcmp(key, "large_query_pairs")) *value = g->large_pairs;
    else if (!strcmp(key, "large_query_slots")) *value = g->large_slots;
    else if (!strcmp(key, "serve_stack_min")) *value = g->serve_stack_min;
    else if (!strcmp(key, "serve_group_wait_us")) *value = g->serve_group_wait_us;
    else if (!strcmp(key, "rare_end_max")) *value = g->rare_end_max;
    else if (!strcmp(key, "serve_lanes")) *value = g->serve_lanes;
    else if (!strcmp(key, "serve_promote_pairs")) *value = g->serve_promote_pairs;
    else if (!strcmp(key, "cooperative_launch")) *value = g->coop_launch ? 1 : 0;
    else if (!strcmp(key, "grid")) *value = g->grid_override;
    else return fail(RPQ_ENOTFOUND, "rpq_get_option: unknown key '%s'", key);
    return RPQ_OK;
}

// ------------------------------------------------------------------ plain query
static int word_width(int32_t Q) { return Q <= 8 ? 1 : Q <= 16 ? 2 : 4; }

// Levels per replay of a captured level graph.
constexpr int GRAPH_LEVELS_PER_REPLAY = 16;

// RPQ_GRAPH_LEVELS: the host loop's phases captured once per graph handle
// (and state-word width and grid) as a HIP graph of GRAPH_LEVELS_PER_REPLAY
// levels that reads the query's Params from device memory; each replay
// advances up to that many levels, and the host checks for the end once per
// replay instead of once per level. Writes the level count to *nlev and
// runs the extract phase.
static rpq_status run_graph_levels(rpq_graph *g, Params &p, int W, bool has_start, hipStream_t s, uint32_t *nlev) {
    const int grid = g->grid_override ? g->grid_override : 1024;
    if (!g->gctl) {
        if (dev_alloc(g, reinterpret_cast<void **>(&g->gctl), 64, "level control") != RPQ_OK ||
            dev_alloc(g, reinterpret_cast<void **>(&g->pdev), sizeof(Params), "params") != RPQ_OK)
            return RPQ_ENOMEM;
    }
    p.st.gctl = g->gctl;
    HIP_TRY(launch_init(W, p, s));
    HIP_TRY(launch_fill(g->gctl, 16, 0, s));
    // the Params block goes up through pinned staging (beyond the status
    // words and the first level records; the copy completes before the first
    // replay is waited for)
    static_assert(sizeof(Params) <= 1024, "params staging");
    uint8_t *stage = g->pinned + g->qconst_cap;
    memcpy(stage + 2688, &p, sizeof(Params));
    HIP_TRY(hipMemcpyAsync(g->pdev, stage + 2688, sizeof(Params), hipMemcpyHostToDevice, s));
    hipGraphExec_t &ex = g->lgraph[W];
    if (ex && g->lgraph_grid[W] != grid) {
        (void)hipGraphExecDestroy(ex);
        ex = nullptr;
    }
    if (!ex) {
        if (!g->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int k = 0; k < GRAPH_LEVELS_PER_REPLAY && e == hipSuccess; k++)
            e = launch_level_g(W, g->pdev, grid, g->cap_stream);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(g->cap_stream, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(e != hipSuccess ? e : e2, "capturing the level graph");
        }
        e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            ex = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        g->lgraph_grid[W] = grid;
    }
    *nlev = 0;
    if (has_start) {
        uint32_t *gc = reinterpret_cast<uint32_t *>(stage + 3712);
        // levels are bounded by |Q| |V| (App. A); a replay count beyond that
        // means the device words are wrong
        const uint64_t cap = (static_cast<uint64_t>(MAX_STATES) * static_cast<uint64_t>(g->V)) / GRAPH_LEVELS_PER_REPLAY + 2;
        for (uint64_t r = 0;; r++) {
            TraceRange tr_("replay of levels from %lld", static_cast<long long>(r * GRAPH_LEVELS_PER_REPLAY));
            HIP_TRY(hipGraphLaunch(ex, s));
            HIP_TRY(hipMemcpyAsync(gc, g->gctl, 16, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (gc[1]) {
                *nlev = gc[2];
                break;
            }
            if (r > cap) return fail(RPQ_EDEVICE, "level graph did not terminate");
        }
    }
    HIP_TRY(launch_final(W, p, *nlev, grid, s));
    return RPQ_OK;
}

rpq_status rpq::run_single(rpq_graph *g, const rpq_nfa *n, int32_t source, uint64_t *out, uint32_t flags,
                           rpq_stats *stats, const SingleExtra *ex) {
    hipStream_t s = g->user_stream ? g->user_stream : g->stream;
    const int W = word_width(n->Q);
    if (g->dirty) {
        const size_t words = (4 * static_cast<size_t>(g->V) + 256) / 4;
        HIP_TRY(launch_fill(g->sv.P, words, 0, s));
        HIP_TRY(launch_fill(g->sv.M[0], words, 0, s));
        HIP_TRY(launch_fill(g->sv.M[1], words, 0, s));
        g->dirty = false;
    }
    g->dirty = true;  // until this query completes
    const uint32_t force = (flags & RPQ_FORCE_PUSH) ? 1u : (flags & RPQ_FORCE_PULL) ? 2u : 0u;
    const uint32_t counters = (flags & RPQ_COUNTERS) ? 1u : 0u;
    // query constants: from the device cache, else built and uploaded into it
    if (g->q_serial != n->serial || g->q_force != force || g->q_counters != counters ||
        g->q_alpha != g->pull_alpha || g->q_beta != g->pull_beta) {
        auto it = g->qcache.find(n->serial);
        if (it != g->qcache.end() && (it->second.force != force || it->second.counters != counters ||
                                      it->second.alpha != g->pull_alpha || it->second.beta != g->pull_beta)) {
            g->qcache.erase(it);
            it = g->qcache.end();
        }
        if (it != g->qcache.end()) {
            g->qv = query_view(g->qconst_dev + it->second.off, it->second.nsym);
        } else {
            int32_t nsym = 0;
            const size_t sz = build_qconst(g, n, force, counters, g->qbuf, &nsym);
            if (nsym > MAX_SYMS) return fail(RPQ_EINVAL, "query uses %d symbols; the limit is %d", nsym, MAX_SYMS);
            if (sz > g->qconst_cap) return fail(RPQ_EINVAL, "query constants too large");
            const size_t need = (sz + 255) & ~static_cast<size_t>(255);
            if (g->qarena_used + need > QARENA_BYTES) {
                // full: start over (every call is complete before the next
                // begins, so no launch still reads the old entries)
                g->qcache.clear();
                g->qarena_used = 0;
            }
            const size_t off = g->qarena_used;
            g->qarena_used += need;
            memcpy(g->pinned, g->qbuf.data(), sz);
            HIP_TRY(hipMemcpyAsync(g->qconst_dev + off, g->pinned, sz, hipMemcpyHostToDevice, s));
            g->qcache[n->serial] = rpq_graph::QEntry{force, counters, g->pull_alpha, g->pull_beta, off, nsym};
            g->qv = query_view(g->qconst_dev + off, nsym);
        }
        g->q_serial = n->serial;
        g->q_force = force;
        g->q_counters = counters;
        g->q_alpha = g->pull_alpha;
        g->q_beta = g->pull_beta;
        // no wait here: nothing else writes this staging area before the
        // synchronisation at the end of the query
    }
    Params p;
    p.g = g->gv;
    p.qv = g->qv;
    p.st = g->sv;
    // barriers in turn; the status words live in this launch's barrier
    p.st.bar = g->bars[g->bar_idx];
    p.st.bar_next = g->bars[g->bar_idx ^ 1];
    p.st.status = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(p.st.bar) + offsetof(GridBarrier, status));
    if (g->bars_dirty) {
        for (GridBarrier *b : g->bars) HIP_TRY(launch_fill(reinterpret_cast<uint32_t *>(b), sizeof(GridBarrier) / 4, 0, s));
        g->bars_dirty = false;
    }
    p.st.out = (flags & RPQ_OUT_DEVICE) ? out : g->dev_out;
    p.source = source;
    p.nsrc = 0;
    p.srcset = nullptr;
    p.dist = nullptr;
    if (ex) {
        p.dist = ex->dist;
        if (ex->nsrc > 0) {
            // the start set's vertices go up on this stream before the launch
            // (the staging buffer is not written again before the call ends)
            HIP_TRY(hipMemcpyAsync(g->dev_srcset, g->pin_srcset, 4 * static_cast<size_t>(ex->nsrc),
                                   hipMemcpyHostToDevice, s));
            p.nsrc = static_cast<uint32_t>(ex->nsrc);
            p.srcset = g->dev_srcset;
        }
    }
    const bool timing = (flags & RPQ_KERNEL_TIMING) != 0;
    int grid_p = g->pgrid[W];
    if (g->plain_grid) grid_p = std::min(g->plain_grid, grid_p);
    if (g->grid_override) grid_p = std::min(g->grid_override, grid_p);
    // the whole call's events are skipped when the kernel itself is timed
    // (device_ms is then the persistent kernel's time)
    const bool whole = !(timing && !(flags & RPQ_HOST_LOOP) && grid_p > 0);
    if (whole) HIP_TRY(hipEventRecord(g->ev[0], s));
    uint32_t nlev = 0;
    float expand_ms = 0.f;
    int32_t launches = 0;
    const bool graph_levels = (flags & RPQ_GRAPH_LEVELS) != 0;
    const bool persistent = !(flags & (RPQ_HOST_LOOP | RPQ_GRAPH_LEVELS)) && grid_p > 0;
    p.st.hstat = nullptr;
    p.st.hserial = 0;
    if (persistent) {
        // the kernel writes its status words to pinned host memory: no copy
        // back in the common case (the flags are cleared before the launch
        // is enqueued; the kernel only ever sets them)
        if (++g->hserial == 0) g->hserial = 1;
        g->hstat[3] = 0;
        g->hstat[6] = 0;
        g->hstat[7] = 0;
        p.st.hstat = g->hstat_dev;
        p.st.hserial = g->hserial;
    }
    PersistentHold hold;  // released when this call returns, after the synchronisation below
    if (persistent) {
        const rpq_status hs = hold.acquire(g->device, grid_p, occupancy_blocks_per_cu(W));
        if (hs != RPQ_OK) return hs;
        g->bar_idx ^= 1;  // the next persistent launch uses the barrier this one zeroes
        if (timing) HIP_TRY(hipEventRecord(g->ev[2], s));
        HIP_TRY(launch_persistent(W, p, grid_p, g->coop_launch, s));
        if (timing) HIP_TRY(hipEventRecord(g->ev[3], s));
        launches = 1;
    } else if (graph_levels) {
        const rpq_status r = run_graph_levels(g, p, W, n->smask != 0, s, &nlev);
        if (r != RPQ_OK) return r;
    } else {
        const int grid = g->grid_override ? g->grid_override : 1024;
        HIP_TRY(launch_init(W, p, s));
        uint32_t *nq_host = reinterpret_cast<uint32_t *>(g->pinned + g->qconst_cap);
        nlev = (n->smask != 0) ? 1u : 0u;
        for (uint32_t lev = 0; nlev > lev; lev++) {
            TraceRange tr_("level %lld", static_cast<long long>(lev));
            HIP_TRY(launch_select(W, p, lev, grid, s));
            if (timing) HIP_TRY(hipEventRecord(g->ev[2], s));
            HIP_TRY(launch_expand(W, p, lev, grid, s));
            if (timing) HIP_TRY(hipEventRecord(g->ev[3], s));
            HIP_TRY(hipMemcpyAsync(nq_host, &p.st.rec[(lev + 1) % REC_RING].nq, 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (timing) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, g->ev[2], g->ev[3]));
                expand_ms += ms;
                launches++;
            }
            if (*nq_host) nlev = lev + 2;
        }
        HIP_TRY(launch_final(W, p, nlev, grid, s));
    }
    if (whole) HIP_TRY(hipEventRecord(g->ev[1], s));
    // results
    uint8_t *stage = g->pinned + g->qconst_cap;
    uint32_t *status = reinterpret_cast<uint32_t *>(stage);
    uint64_t *cnt = reinterpret_cast<uint64_t *>(stage + 64);
    // status words 0..6 and the abort flag in one copy; the first per-level
    // records with them (most queries have fewer levels), the rest below
    static_assert(offsetof(GridBarrier, abort) == offsetof(GridBarrier, status) + 28, "abort follows status");
    constexpr uint32_t LVL_SPEC = 64;
    uint64_t *lp = reinterpret_cast<uint64_t *>(stage + 128);
    if (!persistent) HIP_TRY(hipMemcpyAsync(status, p.st.status, 32, hipMemcpyDeviceToHost, s));
    if (counters) HIP_TRY(hipMemcpyAsync(cnt, p.st.cnt, 32, hipMemcpyDeviceToHost, s));
    // without per-level outputs the persistent kernel's status words carry |P|
    const bool need_lvl = stats && (stats->level_cap > 0 || !persistent);
    if (need_lvl) HIP_TRY(hipMemcpyAsync(lp, p.st.lvl, 8 * LVL_STRIDE * LVL_SPEC, hipMemcpyDeviceToHost, s));
    if (!(flags & RPQ_OUT_DEVICE))
        HIP_TRY(hipMemcpyAsync(out, g->dev_out, 8 * g->nwords, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (persistent) {
        const volatile uint32_t *h = g->hstat;
        if (h[3] || h[6] || h[7] != g->hserial) {
            // a violation, an abort or no final status: the device's own
            // words (the violation count, the barrier's abort flag)
            HIP_TRY(hipMemcpy(status, p.st.status, 32, hipMemcpyDeviceToHost));
            if (h[6]) status[7] = 1;
            if (h[3] && !status[3]) status[3] = 1;
            if (h[7] != g->hserial && !status[7] && !status[3])
                return fail(RPQ_EDEVICE, "persistent traversal ended without its status");
        } else {
            for (int k = 0; k < 8; k++) status[k] = h[k];
            status[3] = 0;
            status[7] = 0;
        }
    }
    if (status[7] && persistent) {
        g->bars_dirty = true;
        return fail(RPQ_EDEVICE, "persistent traversal aborted: grid barrier timed out");
    }
    if (status[3]) return fail(RPQ_EDEVICE, "internal invariant violated %u times (index out of range)", status[3]);
    const uint32_t levels = persistent ? status[0] : nlev;
    if (stats) {
        stats->levels = static_cast<int32_t>(levels);
        stats->push_levels = static_cast<int32_t>(status[1]);
        stats->pull_levels = static_cast<int32_t>(status[2]);
        stats->batch = 1;
        if (timing && launches == 1 && !(flags & RPQ_HOST_LOOP)) {
            HIP_TRY(hipEventElapsedTime(&expand_ms, g->ev[2], g->ev[3]));
        }
        float ms = expand_ms;
        if (whole) HIP_TRY(hipEventElapsedTime(&ms, g->ev[0], g->ev[1]));
        stats->device_ms = ms;
        stats->expand_ms = timing ? expand_ms : 0.0;
        stats->expand_launches = timing ? launches : 0;
        if (need_lvl) {
            const uint32_t ncopy = std::min<uint32_t>(levels + 1, LVL_COUNT_CAP);
            if (ncopy > LVL_SPEC)
                HIP_TRY(hipMemcpy(lp + LVL_STRIDE * LVL_SPEC, p.st.lvl + LVL_STRIDE * LVL_SPEC,
                                  8 * LVL_STRIDE * static_cast<size_t>(ncopy - LVL_SPEC), hipMemcpyDeviceToHost));
            stats->visited_pairs = stats_levels(stats, lp, ncopy, levels);
        } else {
            stats->visited_pairs = static_cast<int64_t>(status[4]) | (static_cast<int64_t>(status[5]) << 32);
        }
        if (counters) {
            const int64_t w = W;
            stats->product_edges = static_cast<int64_t>(cnt[0]);
            stats->scans = static_cast<int64_t>(cnt[1]);
            stats->scanned_edges = static_cast<int64_t>(cnt[2]);
            stats->active = static_cast<int64_t>(cnt[3]);
            stats->alg_bytes = (2 * w + 8) * stats->active + 8 * stats->scans + (4 + w) * stats->scanned_edges +
                               (static_cast<int64_t>(g->V) + 7) / 8;
        }
    }
    g->dirty = false;
    return RPQ_OK;
}

static void reverse_nfa(const rpq_nfa *n, rpq_nfa &rev);

// The rare-end plan (the evaluation-order hybrid Sec. 5.5 and Sec. 6 call
// for on rare labels). A walk the NFA accepts ends either at the source
// (the zero-length walk, when a start state is final) or with a step into a
// final state, so every answer vertex other than the source is an endpoint
// of an edge under a symbol of some transition into a final state: the
// candidates T. When T is small, the answer is the candidates t from which
// the reversed automaton reaches the source (t in SSR(s, R) iff s in
// SSR(t, R reversed)), found by one stacked traversal from all of T that
// only reports, per candidate, whether the source was reached in a final
// state. The answer is identical to the forward traversal's.
// Sets *used when the plan ran; returns an error only when it was forced and
// does not apply, or when it failed.
static rpq_status rare_end(rpq_graph *g, const rpq_nfa *n, int32_t source, uint64_t *out, uint32_t flags,
                           rpq_stats *stats, bool *used) {
    *used = false;
    const bool forced = (flags & RPQ_RARE_END) != 0;
    const int64_t limit = forced ? MAX_BATCH : std::min<int64_t>(g->rare_end_max, MAX_BATCH);
    if (limit <= 0) return RPQ_OK;
    const uint32_t excl = RPQ_HOST_LOOP | RPQ_GRAPH_LEVELS | RPQ_COUNTERS | RPQ_FORCE_PUSH | RPQ_FORCE_PULL;
    if ((flags & excl) || (stats && stats->level_cap > 0)) {
        if (forced)
            return fail(RPQ_EINVAL, "rpq_single_source: RPQ_RARE_END excludes per-level outputs, counters and "
                                    "direction or level-driver flags");
        return RPQ_OK;
    }
    const int32_t L = g->L;
    // (direction, label) whose rows are the candidate endpoints
    std::vector<uint64_t> parts;
    int64_t total = 0;
    for (const Trans &t : n->trans) {
        if (!((n->fmask >> t.to) & 1u)) continue;
        const bool inv = t.sym >= n->NL;
        const int32_t lab = inv ? t.sym - n->NL : t.sym;
        if (lab >= L || g->label_edges[lab] == 0) continue;
        // a step with label l ends at the head of an l-edge (a row of the
        // transposed direction); with its inverse at the tail (a row of G^l)
        const uint64_t key = static_cast<uint64_t>(inv ? OUT : IN) * L + lab;
        if (std::find(parts.begin(), parts.end(), key) != parts.end()) continue;
        parts.push_back(key);
        total += g->label_rows[inv ? OUT : IN][lab];
    }
    if (total > limit) {
        if (forced)
            return fail(RPQ_EINVAL, "rpq_single_source: %lld candidate endpoints exceed the %d of RPQ_RARE_END",
                        (long long)total, MAX_BATCH);
        return RPQ_OK;
    }
    hipStream_t s = g->user_stream ? g->user_stream : g->stream;
    std::vector<int32_t> cand(static_cast<size_t>(total));
    size_t at = 0;
    for (uint64_t key : parts) {
        const int dir = static_cast<int>(key / L);
        const int32_t lab = static_cast<int32_t>(key % L);
        const int64_t rows = g->label_rows[dir][lab];
        if (rows)
            HIP_TRY(hipMemcpy(cand.data() + at, g->gv.rowvert + g->rbase[key], 4 * static_cast<size_t>(rows),
                              hipMemcpyDeviceToHost));
        at += static_cast<size_t>(rows);
    }
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    for (int32_t v : cand)
        if (v < 0 || v >= g->V) return fail(RPQ_EDEVICE, "rpq_single_source: corrupt row vertex %d", v);
    std::vector<uint64_t> ans(static_cast<size_t>(g->nwords), 0ull);
    rpq_stats st2{};
    if (!cand.empty()) {
        rpq_nfa rev;
        reverse_nfa(n, rev);
        uint64_t hit[MAX_BATCH / 64];
        const rpq_status r = stacked_run(g, &rev, cand.data(), static_cast<int32_t>(cand.size()), hit, 0, &st2,
                                         "rpq_single_source (rare-end plan)", nullptr, source);
        if (r != RPQ_OK) return r;
        for (size_t i = 0; i < cand.size(); i++)
            if ((hit[i >> 6] >> (i & 63)) & 1ull) ans[static_cast<size_t>(cand[i]) >> 6] |= 1ull << (cand[i] & 63);
    }
    if (n->smask & n->fmask) ans[static_cast<size_t>(source) >> 6] |= 1ull << (source & 63);
    if (flags & RPQ_OUT_DEVICE) {
        HIP_TRY(hipMemcpyAsync(out, ans.data(), 8 * ans.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        memcpy(out, ans.data(), 8 * ans.size());
    }
    if (stats) {
        stats_reset(stats);
        stats->levels = st2.levels;
        stats->push_levels = st2.push_levels;
        stats->pull_levels = st2.pull_levels;
        stats->visited_pairs = st2.visited_pairs;
        stats->device_ms = st2.device_ms;
        stats->expand_ms = st2.expand_ms;
        stats->expand_launches = st2.expand_launches;
        stats->batch = static_cast<int32_t>(cand.size());
        stats->plan = 1;
    }
    *used = true;
    return RPQ_OK;
}

rpq_status rpq_single_source(rpq_graph *g, const rpq_nfa *n, int32_t source, uint64_t *out_bitmap,
                             uint32_t flags, rpq_stats *stats) {
    TraceRange tr_("rpq_single_source");
    if (!g || !n || !out_bitmap) return fail(RPQ_EINVAL, "rpq_single_source: NULL argument");
    if (source < 0 || source >= g->V)
        return fail(RPQ_EINVAL, "rpq_single_source: source %d outside [0, %d)", source, g->V);
    if ((flags & RPQ_FORCE_PUSH) && (flags & RPQ_FORCE_PULL))
        return fail(RPQ_EINVAL, "rpq_single_source: RPQ_FORCE_PUSH and RPQ_FORCE_PULL together");
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    HIP_TRY(hipSetDevice(g->device));
    bool used = false;
    const rpq_status r = rare_end(g, n, source, out_bitmap, flags, stats, &used);
    if (r != RPQ_OK || used) return r;
    return run_single(g, n, source, out_bitmap, flags & ~RPQ_RARE_END, stats);
}

// Single-destination reachability (Sec. 2, the SDR map; Sec. 4 evaluates it
// as the single-source query of the reversed automaton): every transition
// turned around with its symbol inverted (a walk read backwards crosses each
// edge the other way), start and final sets swapped.
// The reversed automaton (reading of Sec. 4's reversal with a two-way
// alphabet): every transition turned around with its symbol inverted (a walk
// read backwards crosses each edge the other way), start and final sets
// swapped.
static void reverse_nfa(const rpq_nfa *n, rpq_nfa &rev) {
    rev.Q = n->Q;
    rev.NL = n->NL;
    rev.smask = n->fmask;
    rev.fmask = n->smask;
    rev.serial = n->serial | (1ull << 63);  // the reversal of n, cached under its own key
    rev.trans.clear();
    rev.trans.reserve(n->trans.size());
    for (const Trans &t : n->trans) {
        const int32_t inv = t.sym < n->NL ? t.sym + n->NL : t.sym - n->NL;
        rev.trans.push_back({inv, t.to, t.from});
    }
}

rpq_status rpq_single_destination(rpq_graph *g, const rpq_nfa *n, int32_t target, uint64_t *out_bitmap,
                                  uint32_t flags, rpq_stats *stats) {
    TraceRange tr_("rpq_single_destination");
    if (!g || !n || !out_bitmap) return fail(RPQ_EINVAL, "rpq_single_destination: NULL argument");
    if (target < 0 || target >= g->V)
        return fail(RPQ_EINVAL, "rpq_single_destination: target %d outside [0, %d)", target, g->V);
    if ((flags & RPQ_FORCE_PUSH) && (flags & RPQ_FORCE_PULL))
        return fail(RPQ_EINVAL, "rpq_single_destination: RPQ_FORCE_PUSH and RPQ_FORCE_PULL together");
    rpq_nfa rev;
    reverse_nfa(n, rev);
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    HIP_TRY(hipSetDevice(g->device));
    return run_single(g, &rev, target, out_bitmap, flags, stats);
}

// Lengths of the shortest accepted walks (the future-work semirings of Sec. 6,
// min over walk lengths in place of the Boolean OR): the same traversal, with
// each vertex's first level that reaches it in a final state recorded by the
// select (by the FIFO-level invariant of App. A that level is the length).
rpq_status rpq_single_source_lengths(rpq_graph *g, const rpq_nfa *n, int32_t source, int32_t *out_lengths,
                                     uint32_t flags, rpq_stats *stats) {
    TraceRange tr_("rpq_single_source_lengths");
    if (!g || !n || !out_lengths) return fail(RPQ_EINVAL, "rpq_single_source_lengths: NULL argument");
    if (source < 0 || source >= g->V)
        return fail(RPQ_EINVAL, "rpq_single_source_lengths: source %d outside [0, %d)", source, g->V);
    if ((flags & RPQ_FORCE_PUSH) && (flags & RPQ_FORCE_PULL))
        return fail(RPQ_EINVAL, "rpq_single_source_lengths: RPQ_FORCE_PUSH and RPQ_FORCE_PULL together");
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    HIP_TRY(hipSetDevice(g->device));
    const bool dev = (flags & RPQ_OUT_DEVICE) != 0;
    if (!dev && !g->dev_dist) {
        const rpq_status st = dev_alloc(g, reinterpret_cast<void **>(&g->dev_dist), 4 * static_cast<size_t>(g->V), "lengths");
        if (st != RPQ_OK) return st;
    }
    SingleExtra ex;
    ex.dist = dev ? out_lengths : g->dev_dist;
    const rpq_status r = run_single(g, n, source, g->dev_out, flags | RPQ_OUT_DEVICE, stats, &ex);
    if (r != RPQ_OK) return r;
    if (!dev) {
        hipStream_t s = g->user_stream ? g->user_stream : g->stream;
        HIP_TRY(hipMemcpyAsync(out_lengths, g->dev_dist, 4 * static_cast<size_t>(g->V), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return RPQ_OK;
}

// Reachability from a set of sources (Def. 2.6 with a start set V_s): the
// traversal starts from M_0 = Q_S x V_s, and F P is the union of the sources'
// single-source answers.
rpq_status rpq_source_set(rpq_graph *g, const rpq_nfa *n, const int32_t *sources, int32_t n_sources,
                          uint64_t *out_bitmap, uint32_t flags, rpq_stats *stats) {
    TraceRange tr_("rpq_source_set");
    if (!g || !n || !sources || !out_bitmap) return fail(RPQ_EINVAL, "rpq_source_set: NULL argument");
    if (n_sources < 1) return fail(RPQ_EINVAL, "rpq_source_set: n_sources < 1");
    for (int32_t i = 0; i < n_sources; i++)
        if (sources[i] < 0 || sources[i] >= g->V)
            return fail(RPQ_EINVAL, "rpq_source_set: source %d outside [0, %d)", sources[i], g->V);
    if ((flags & RPQ_FORCE_PUSH) && (flags & RPQ_FORCE_PULL))
        return fail(RPQ_EINVAL, "rpq_source_set: RPQ_FORCE_PUSH and RPQ_FORCE_PULL together");
    // distinct vertices: the level-0 queue holds each start vertex once
    std::vector<int32_t> vs(sources, sources + n_sources);
    std::sort(vs.begin(), vs.end());
    vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    HIP_TRY(hipSetDevice(g->device));
    if (!g->dev_srcset) {
        const rpq_status st = dev_alloc(g, reinterpret_cast<void **>(&g->dev_srcset), 4 * static_cast<size_t>(g->V), "start set");
        if (st != RPQ_OK) return st;
    }
    if (!g->pin_srcset) HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&g->pin_srcset), 4 * static_cast<size_t>(g->V), hipHostMallocDefault));
    memcpy(g->pin_srcset, vs.data(), 4 * vs.size());
    SingleExtra ex;
    ex.nsrc = static_cast<int32_t>(vs.size());
    return run_single(g, n, vs[0], out_bitmap, flags, stats, &ex);
}
