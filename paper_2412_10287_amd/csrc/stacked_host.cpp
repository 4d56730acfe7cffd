// rpq_multi_source: sources under one NFA evaluated together by the stacked
// kernel (stacked.hip), in batches of at most max_batch sources.
#include <string.h>

#include <algorithm>

#include "api_internal.h"
#include "trace.h"
#include "stacked.h"

using namespace rpq;

namespace rpq {

struct BatchState {
    std::vector<void *> allocs;
    uint64_t state_words = 0;  // capacity of P / M arrays (uint64 words)
    StackParams p{};
    uint8_t *qconst = nullptr;
    size_t qconst_cap = 0;
    uint64_t *out = nullptr;  // internal output (host-memory results)
    int64_t out_words = 0;
    int32_t *sources = nullptr;  // device copy of one batch's sources (MAX_BATCH entries)
    uint8_t *pinned = nullptr;
    int grid[2][17] = {{0}};  // [QM == 32][G]
};

}  // namespace rpq

#define BT(call)                                                  \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return hip_fail(e_, #call);         \
    } while (0)

static void free_batch(BatchState *b) {
    if (!b) return;
    for (void *x : b->allocs) (void)hipFree(x);
    if (b->pinned) (void)hipHostFree(b->pinned);
    delete b;
}

void rpq::batch_free(rpq_graph *g) {
    free_batch(g->batch);
    g->batch = nullptr;
}

static rpq_status balloc(BatchState *b, void **p, size_t bytes, const char *what) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 64);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(RPQ_ENOMEM, "rpq_multi_source: hipMalloc(%s, %zu bytes): %s", what, bytes, hipGetErrorString(e));
    }
    b->allocs.push_back(*p);
    return RPQ_OK;
}

// (Re)allocates the stacked state for rows of Q*G words, zeroed.
static rpq_status batch_prepare(rpq_graph *g, int32_t Q, int G, int32_t B, hipStream_t s) {
    const uint64_t need = static_cast<uint64_t>(g->V) * Q * G + 64;
    BatchState *b = g->batch;
    if (b && b->state_words >= need && b->out_words >= static_cast<int64_t>(B) * g->nwords) return RPQ_OK;
    batch_free(g);
    b = g->batch = new (std::nothrow) BatchState;
    if (!b) return fail(RPQ_ENOMEM, "rpq_multi_source: out of host memory");
    rpq_status st;
    StackParams &p = b->p;
    const uint64_t words = need;
    b->state_words = words;
    if ((st = balloc(b, reinterpret_cast<void **>(&p.P), 8 * words, "P")) != RPQ_OK) return st;
    if ((st = balloc(b, reinterpret_cast<void **>(&p.M[0]), 8 * words, "M")) != RPQ_OK) return st;
    if ((st = balloc(b, reinterpret_cast<void **>(&p.M[1]), 8 * words, "M")) != RPQ_OK) return st;
    for (int k = 0; k < 2; k++) {
        if ((st = balloc(b, reinterpret_cast<void **>(&p.sup[k]), 4 * static_cast<size_t>(g->V) + 64, "sup")) != RPQ_OK)
            return st;
        if ((st = balloc(b, reinterpret_cast<void **>(&p.q[k]), 4 * static_cast<size_t>(g->V) + 64, "queue")) != RPQ_OK)
            return st;
    }
    p.item_cap = static_cast<uint64_t>(g->rows[OUT] + g->rows[IN]) + 1;
    for (uint32_t **a : {&p.it_ebase, &p.it_beg, &p.it_v, &p.it_u, &p.it_s})
        if ((st = balloc(b, reinterpret_cast<void **>(a), 4 * p.item_cap, "items")) != RPQ_OK) return st;
    p.tile_cap = (2 * static_cast<uint64_t>(g->E)) / (TILE / 16) + 2;
    if ((st = balloc(b, reinterpret_cast<void **>(&p.tile_first), 4 * p.tile_cap, "tiles")) != RPQ_OK) return st;
    if ((st = balloc(b, reinterpret_cast<void **>(&p.rec), sizeof(LevelRec) * REC_RING, "rec")) != RPQ_OK) return st;
    if ((st = balloc(b, reinterpret_cast<void **>(&p.bar), sizeof(GridBarrier), "barrier")) != RPQ_OK) return st;
    if ((st = balloc(b, reinterpret_cast<void **>(&p.status), 64, "status")) != RPQ_OK) return st;
    if ((st = balloc(b, reinterpret_cast<void **>(&p.cnt), 64, "counters")) != RPQ_OK) return st;
    if ((st = balloc(b, reinterpret_cast<void **>(&p.hand), 4 * HAND_WORDS, "hand-off words")) != RPQ_OK) return st;
    if ((st = balloc(b, reinterpret_cast<void **>(&p.lvl), 8 * LVL_STRIDE * (LVL_COUNT_CAP + 1), "lvl")) != RPQ_OK)
        return st;
    if ((st = balloc(b, reinterpret_cast<void **>(&b->sources), 4 * static_cast<size_t>(MAX_BATCH), "sources")) !=
        RPQ_OK)
        return st;
    b->qconst_cap = g->qconst_cap;
    if ((st = balloc(b, reinterpret_cast<void **>(&b->qconst), b->qconst_cap, "qconst")) != RPQ_OK) return st;
    b->out_words = static_cast<int64_t>(std::max<int32_t>(B, g->max_batch)) * g->nwords;
    if ((st = balloc(b, reinterpret_cast<void **>(&b->out), 8 * static_cast<size_t>(b->out_words), "out")) != RPQ_OK)
        return st;
    BT(hipHostMalloc(reinterpret_cast<void **>(&b->pinned), b->qconst_cap + 4096 + 8 * LVL_COUNT_CAP,
                     hipHostMallocDefault));
    for (uint64_t *a : {p.P, p.M[0], p.M[1]}) BT(launch_fill(reinterpret_cast<uint32_t *>(a), 2 * words, 0, s));
    for (int k = 0; k < 2; k++) BT(launch_fill(p.sup[k], static_cast<uint64_t>(g->V) + 16, 0, s));
    for (int G2 : {1, 2, 4, 8, 16}) {
        b->grid[0][G2] = stacked_grid(G2, 8);
        b->grid[1][G2] = stacked_grid(G2, 32);
    }
    BT(hipStreamSynchronize(s));
    return RPQ_OK;
}

// Lays out one batch's device state for rows of Q*G words inside an arena at
// `base` (nullptr: sizes only): the arrays of StackParams, the query
// constants, the batch's sources and its result bitmaps, each 256-byte
// aligned. Returns the bytes needed.
size_t rpq::stacked_arena_layout(const rpq_graph *g, int32_t Q, int G, int32_t B, uint8_t *base, StackParams *p,
                                 uint8_t **qconst, int32_t **srcs, uint64_t **out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *r = base ? static_cast<void *>(base + off) : nullptr;
        off += (bytes + 255) & ~static_cast<size_t>(255);
        return r;
    };
    const uint64_t words = static_cast<uint64_t>(g->V) * Q * G + 64;
    StackParams q{};
    q.P = static_cast<uint64_t *>(take(8 * words));
    q.M[0] = static_cast<uint64_t *>(take(8 * words));
    q.M[1] = static_cast<uint64_t *>(take(8 * words));
    for (int k = 0; k < 2; k++) {
        q.sup[k] = static_cast<uint32_t *>(take(4 * static_cast<size_t>(g->V) + 64));
        q.q[k] = static_cast<int32_t *>(take(4 * static_cast<size_t>(g->V) + 64));
    }
    q.item_cap = static_cast<uint64_t>(g->rows[OUT] + g->rows[IN]) + 1;
    for (uint32_t **a : {&q.it_ebase, &q.it_beg, &q.it_v, &q.it_u, &q.it_s}) *a = static_cast<uint32_t *>(take(4 * q.item_cap));
    q.tile_cap = (2 * static_cast<uint64_t>(g->E)) / (TILE / 16) + 2;
    q.tile_first = static_cast<uint32_t *>(take(4 * q.tile_cap));
    q.rec = static_cast<LevelRec *>(take(sizeof(LevelRec) * REC_RING));
    q.bar = static_cast<GridBarrier *>(take(sizeof(GridBarrier)));
    q.status = static_cast<uint32_t *>(take(64));
    q.cnt = static_cast<uint64_t *>(take(64));
    q.hand = static_cast<uint32_t *>(take(4 * HAND_WORDS));
    q.lvl = static_cast<uint64_t *>(take(8 * LVL_STRIDE * (LVL_COUNT_CAP + 1)));
    uint8_t *qc = static_cast<uint8_t *>(take(g->qconst_cap));
    int32_t *sv = static_cast<int32_t *>(take(4 * static_cast<size_t>(MAX_BATCH)));
    uint64_t *ob = static_cast<uint64_t *>(take(8 * static_cast<size_t>(B) * g->nwords));
    if (base) {
        *p = q;
        *qconst = qc;
        *srcs = sv;
        *out = ob;
    }
    return off;
}

// The stacked traversal of `sources` in batches of at most max_batch. Its
// device state comes from g->batch (allocated or grown here), or, with an
// arena (ar != nullptr), from the arena alone: then nothing is allocated,
// the arena's arrays are cleared before each batch, and the host staging is
// the graph handle's pinned buffer.
// After a launch of the stacked kernel that may stop before a large push
// level: runs such levels with the phase kernels (expansion that marks the
// candidate state sets, vertex-ordered queue, select of the next level), one
// host check per level, and relaunches the persistent kernel where a level
// is small, pulls, or the traversal ends (its final phase runs there). The
// persistent grid keeps its share of the co-resident workgroups throughout
// (the caller holds it). `stage` is 128 bytes of pinned host memory.
static rpq_status st_handoff_loop(rpq_graph *g, StackParams &p, int G, int QM, int grid, const QHeader *qh,
                                  uint8_t *stage, hipStream_t s, const char *who) {
    uint32_t *hw = reinterpret_cast<uint32_t *>(stage);          // hand words (64 bytes)
    uint64_t *rw = reinterpret_cast<uint64_t *>(stage + 64);     // level records' fields
    const uint64_t big = std::max<uint64_t>(p.handoff_edges, static_cast<uint64_t>(g->V) / ST_SWEEP_DIV);
    // levels are bounded by |Q| |V| (App. A); more hand-offs mean a fault
    const uint64_t cap = static_cast<uint64_t>(MAX_STATES) * static_cast<uint64_t>(g->V) + 2;
    for (uint64_t round = 0;; round++) {
        BT(hipMemcpyAsync(hw, p.hand, 4 * HAND_WORDS, hipMemcpyDeviceToHost, s));
        BT(hipStreamSynchronize(s));
        if (hw[HAND_EXIT] != 1) return RPQ_OK;  // finished, or aborted (the caller's status check reports it)
        if (round > cap) return fail(RPQ_EDEVICE, "%s: the level loop did not terminate", who);
        uint32_t lev = hw[HAND_LEVEL], npush = hw[HAND_NPUSH];
        const uint32_t npull = hw[HAND_NPULL];
        bool record = false;  // the persistent kernel recorded the first level
        uint64_t last = 0;
        while (true) {
            BT(launch_st_expand(G, QM, p, lev, record, s));
            BT(launch_st_compact(p, lev, s));
            BT(launch_st_select(G, QM, p, lev + 1, qh->counters != 0, s));
            npush++;
            const LevelRec *rn = &p.rec[(lev + 1) % REC_RING];
            const LevelRec *rc = &p.rec[lev % REC_RING];
            BT(hipMemcpyAsync(&rw[0], &rn->nq, 4, hipMemcpyDeviceToHost, s));
            BT(hipMemcpyAsync(&rw[1], &rn->sel, 8, hipMemcpyDeviceToHost, s));
            BT(hipMemcpyAsync(&rw[2], &rc->pairs, 8, hipMemcpyDeviceToHost, s));
            BT(hipStreamSynchronize(s));
            const uint32_t nq = static_cast<uint32_t>(rw[0]);
            const uint64_t edges = rw[1] & 0xffffffffull;
            last = rw[2];
            lev++;
            // the direction the persistent kernel would take after a push
            // level (st_decide with prev = push)
            const bool pull = QM <= 8 && qh->force != 1 &&
                              (qh->force == 2 || (qh->alpha > 0.f && static_cast<double>(edges) * qh->alpha >
                                                                          static_cast<double>(qh->e_rel)));
            if (nq == 0 || edges < big || pull || lev > cap) break;
            record = true;
        }
        // the persistent kernel continues at level lev, whose select is done
        hw[HAND_EXIT] = 0;
        hw[HAND_LEVEL] = lev;
        hw[HAND_RESUME] = 1;
        hw[HAND_NPUSH] = npush;
        hw[HAND_NPULL] = npull;
        hw[HAND_LAST_LO] = static_cast<uint32_t>(last);
        hw[HAND_LAST_HI] = static_cast<uint32_t>(last >> 32);
        BT(hipMemcpyAsync(p.hand, hw, 4 * HAND_WORDS, hipMemcpyHostToDevice, s));
        BT(launch_fill(reinterpret_cast<uint32_t *>(p.bar), sizeof(GridBarrier) / 4, 0, s));
        BT(launch_stacked(G, QM, p, grid, g->coop_launch, s));
    }
}

rpq_status rpq::stacked_run(rpq_graph *g, const rpq_nfa *n, const int32_t *sources, int32_t n_sources,
                            uint64_t *out_bitmaps, uint32_t flags, rpq_stats *stats, const char *who,
                            const StackArena *ar, int32_t probe) {
    if (!g || !n || !sources || !out_bitmaps) return fail(RPQ_EINVAL, "%s: NULL argument", who);
    if (n_sources < 1) return fail(RPQ_EINVAL, "%s: n_sources < 1", who);
    for (int32_t i = 0; i < n_sources; i++)
        if (sources[i] < 0 || sources[i] >= g->V)
            return fail(RPQ_EINVAL, "%s: source %d outside [0, %d)", who, sources[i], g->V);
    if ((flags & RPQ_FORCE_PUSH) && (flags & RPQ_FORCE_PULL))
        return fail(RPQ_EINVAL, "%s: RPQ_FORCE_PUSH and RPQ_FORCE_PULL together", who);
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    BT(hipSetDevice(g->device));
    hipStream_t s = g->user_stream ? g->user_stream : g->stream;
    if (probe >= 0 && (n_sources > MAX_BATCH || probe >= g->V))
        return fail(RPQ_EINVAL, "%s: a probe needs at most %d sources and a vertex id", who, MAX_BATCH);
    const int32_t maxb = probe >= 0 ? MAX_BATCH : std::min<int32_t>(g->max_batch, MAX_BATCH);
    const uint32_t force = (flags & RPQ_FORCE_PUSH) ? 1u : (flags & RPQ_FORCE_PULL) ? 2u : 0u;
    // automata with at most 8 states use the kernel with byte-sized state sets
    // (which also has the pull direction)
    const int QM = n->Q <= 8 ? 8 : 32;
    // host staging: [0, qconst_cap) query constants, then 4 KB of sources,
    // then status and counter words (128 B), then (arena) the level records
    uint8_t *pin = nullptr;
    size_t lvl_room = 0;
    int32_t nsym = 0;
    size_t qsz = 0;
    std::vector<uint8_t> qbuf;
    if (ar) {
        const int32_t B0 = std::min(maxb, n_sources);
        int G0 = 1;
        while (G0 * 64 < B0) G0 *= 2;
        const size_t need = stacked_arena_layout(g, n->Q, G0, B0, nullptr, nullptr, nullptr, nullptr, nullptr);
        if (need > ar->bytes)
            return fail(RPQ_EINVAL,
                        "%s: %d sources of %d states on %d vertices need %zu bytes of scratch; the limit is %zu", who,
                        B0, n->Q, g->V, need, ar->bytes);
        pin = g->pinned;
        lvl_room = (g->pinned_cap - g->qconst_cap - 4096 - 256) / (8 * LVL_STRIDE);
        qsz = build_qconst_into(g, n, force, (flags & RPQ_COUNTERS) ? 1u : 0u, pin, g->qconst_cap, &nsym);
    } else {
        qsz = build_qconst(g, n, force, (flags & RPQ_COUNTERS) ? 1u : 0u, qbuf, &nsym);
    }
    if (nsym > MAX_SYMS || qsz == 0 || qsz > g->qconst_cap)
        return fail(RPQ_EINVAL, "%s: query uses %d symbols; the limit is %d", who, nsym, MAX_SYMS);
    {
        // the stacked path has its own direction thresholds
        QHeader *h = reinterpret_cast<QHeader *>(ar ? pin : qbuf.data());
        h->alpha = static_cast<float>(g->stack_alpha);
        h->beta = static_cast<float>(g->stack_beta);
    }
    int32_t push_levels = 0, pull_levels = 0;
    int32_t levels = 0;
    int64_t pairs = 0, scans = 0, edges = 0, updates = 0, active = 0, bytes = 0, pedges = 0;
    float total_ms = 0.f;
    std::vector<uint64_t> lvl_host;
    const uint64_t *lvl_rec = nullptr;
    uint32_t lvl_nrec = 0, lvl_levels = 0;
    for (int32_t b0 = 0; b0 < n_sources; b0 += maxb) {
        TraceRange tr_("stacked batch from source %lld", static_cast<long long>(b0));
        const int32_t B = std::min(maxb, n_sources - b0);
        int G = 1;
        while (G * 64 < B) G *= 2;
        StackParams p;
        uint8_t *dq = nullptr;
        int32_t *dsrc = nullptr;
        uint64_t *dout = nullptr;
        int full = 0;
        if (ar) {
            stacked_arena_layout(g, n->Q, G, B, ar->base, &p, &dq, &dsrc, &dout);
            // the arena keeps whatever the last call on this GPU left there
            const uint64_t words = static_cast<uint64_t>(g->V) * n->Q * G + 64;
            for (uint64_t *a : {p.P, p.M[0], p.M[1]}) BT(launch_fill(reinterpret_cast<uint32_t *>(a), 2 * words, 0, s));
            for (int k = 0; k < 2; k++) BT(launch_fill(p.sup[k], static_cast<uint64_t>(g->V) + 16, 0, s));
            full = ar->grid[QM == 8 ? 0 : 1][G];
        } else {
            rpq_status st = batch_prepare(g, n->Q, G, probe >= 0 ? 1 : B, s);
            if (st != RPQ_OK) return st;
            BatchState *bs = g->batch;
            p = bs->p;
            dq = bs->qconst;
            dsrc = bs->sources;
            dout = bs->out;
            pin = bs->pinned;
            memcpy(pin, qbuf.data(), qsz);
            full = bs->grid[QM == 8 ? 0 : 1][G];
        }
        int32_t *hsrc = reinterpret_cast<int32_t *>(pin + g->qconst_cap);
        memcpy(hsrc, sources + b0, 4 * static_cast<size_t>(B));
        BT(hipMemcpyAsync(dq, pin, qsz, hipMemcpyHostToDevice, s));
        BT(hipMemcpyAsync(dsrc, hsrc, 4 * static_cast<size_t>(B), hipMemcpyHostToDevice, s));
        p.g = g->gv;
        p.qv = query_view(dq, nsym);
        p.sources = dsrc;
        p.B = B;
        p.Q = n->Q;
        p.V = g->V;
        p.nwords = g->nwords;
        p.out = (flags & RPQ_OUT_DEVICE) && probe < 0 ? out_bitmaps + static_cast<size_t>(b0) * g->nwords : dout;
        p.probe = probe >= 0 ? static_cast<uint32_t>(probe) : static_cast<uint32_t>(g->V);
        const int grid = g->grid_override ? std::min(g->grid_override, full) : full;
        if (grid <= 0) return fail(RPQ_EDEVICE, "%s: no co-resident grid for the stacked kernel", who);
        BT(launch_fill(reinterpret_cast<uint32_t *>(p.bar), sizeof(GridBarrier) / 4, 0, s));
        // the grid's share of the device's co-resident workgroups (returned
        // after the synchronisation below, at the end of this batch)
        PersistentHold hold;
        {
            const rpq_status hs = hold.acquire(g->device, grid, stacked_blocks_per_cu(G, QM));
            if (hs != RPQ_OK) return hs;
        }
        // large push levels go to the phase kernels (not with a probe, whose
        // traversals are small by construction)
        p.handoff_edges = probe < 0 ? static_cast<uint64_t>(g->stack_handoff) : 0;
        BT(launch_fill(p.hand, HAND_WORDS, 0, s));
        BT(hipEventRecord(g->ev[2], s));
        BT(launch_stacked(G, QM, p, grid, g->coop_launch, s));
        if (p.handoff_edges) {
            const QHeader *qh = reinterpret_cast<const QHeader *>(pin);  // the query constants staged above
            const rpq_status hs = st_handoff_loop(g, p, G, QM, grid, qh, pin + g->qconst_cap + 4096 + 128, s, who);
            if (hs != RPQ_OK) {
                if (!ar) batch_free(g);
                return hs;
            }
        }
        BT(hipEventRecord(g->ev[3], s));
        uint32_t *hst = reinterpret_cast<uint32_t *>(pin + g->qconst_cap + 4 * 1024);
        uint64_t *hcnt = reinterpret_cast<uint64_t *>(pin + g->qconst_cap + 4 * 1024 + 64);
        BT(hipMemcpyAsync(hst, p.status, 16, hipMemcpyDeviceToHost, s));
        BT(hipMemcpyAsync(hcnt, p.cnt, 8 * ST_NCNT, hipMemcpyDeviceToHost, s));
        BT(hipMemcpyAsync(hst + 4, &p.bar->abort, 4, hipMemcpyDeviceToHost, s));
        if (probe >= 0)
            BT(hipMemcpyAsync(out_bitmaps, dout, 8 * static_cast<size_t>((B + 63) / 64), hipMemcpyDeviceToHost, s));
        else if (!(flags & RPQ_OUT_DEVICE))
            BT(hipMemcpyAsync(out_bitmaps + static_cast<size_t>(b0) * g->nwords, dout,
                              8 * static_cast<size_t>(B) * g->nwords, hipMemcpyDeviceToHost, s));
        BT(hipStreamSynchronize(s));
        if (hst[4]) {
            if (!ar) batch_free(g);
            return fail(RPQ_EDEVICE, "%s: traversal aborted (grid barrier timed out)", who);
        }
        if (hst[3]) {
            if (!ar) batch_free(g);
            return fail(RPQ_EDEVICE, "%s: internal invariant violated %u times", who, hst[3]);
        }
        float ms = 0.f;
        BT(hipEventElapsedTime(&ms, g->ev[2], g->ev[3]));
        total_ms += ms;
        levels = std::max<int32_t>(levels, static_cast<int32_t>(hst[0]));
        push_levels += static_cast<int32_t>(hst[1]);
        pull_levels += static_cast<int32_t>(hst[2]);
        // algorithmic bytes of the stacked traversal, levels in lockstep:
        // per active (level, vertex) its queue entry read and written (8 B)
        // and its frontier column read and written (2W, W = 4 B per non-zero
        // 32-bit word of the column over all states and sources); per scan
        // its row-pointer pair (8 B); per scanned edge its 4-byte index and
        // the column's W bytes delivered to the neighbour; and the B result
        // bitmaps
        scans += static_cast<int64_t>(hcnt[ST_CNT_SCANS]);
        edges += static_cast<int64_t>(hcnt[ST_CNT_EDGES]);
        updates += static_cast<int64_t>(hcnt[ST_CNT_UPDATES]);
        active += static_cast<int64_t>(hcnt[ST_CNT_ACTIVE]);
        pedges += static_cast<int64_t>(hcnt[ST_CNT_PE]);
        bytes += 8 * static_cast<int64_t>(hcnt[ST_CNT_ACTIVE]) + 8 * static_cast<int64_t>(hcnt[ST_CNT_SCANS]) +
                 4 * static_cast<int64_t>(hcnt[ST_CNT_EDGES]) + static_cast<int64_t>(hcnt[ST_CNT_WBYTES]) +
                 static_cast<int64_t>(B) * ((static_cast<int64_t>(g->V) + 7) / 8);
        uint32_t nrec = std::min<uint32_t>(hst[0] + 1, LVL_COUNT_CAP);
        if (ar) {
            nrec = std::min<uint32_t>(nrec, static_cast<uint32_t>(lvl_room));
            uint64_t *dst = reinterpret_cast<uint64_t *>(pin + g->qconst_cap + 4096 + 256);
            BT(hipMemcpy(dst, p.lvl, 8 * LVL_STRIDE * static_cast<size_t>(nrec), hipMemcpyDeviceToHost));
            lvl_rec = dst;
        } else {
            lvl_host.assign(static_cast<size_t>(nrec) * LVL_STRIDE, 0);
            BT(hipMemcpy(lvl_host.data(), p.lvl, 8 * lvl_host.size(), hipMemcpyDeviceToHost));
            lvl_rec = lvl_host.data();
        }
        lvl_nrec = nrec;
        lvl_levels = hst[0];
        pairs += stats_levels(nullptr, lvl_rec, nrec, hst[0]);
    }
    if (stats) {
        stats_reset(stats);
        stats_levels(stats, lvl_rec, lvl_nrec, lvl_levels);
        stats->levels = levels;
        stats->push_levels = push_levels;
        stats->pull_levels = pull_levels;
        stats->visited_pairs = pairs;
        stats->batch = std::min(n_sources, maxb);
        stats->device_ms = total_ms;
        stats->expand_ms = total_ms;
        stats->expand_launches = (n_sources + maxb - 1) / maxb;
        stats->updates = updates;
        if (flags & RPQ_COUNTERS) {
            stats->scans = scans;
            stats->scanned_edges = edges;
            stats->active = active;
            stats->alg_bytes = bytes;
            stats->product_edges = pedges;
        }
    }
    return RPQ_OK;
}

rpq_status rpq_multi_source(rpq_graph *g, const rpq_nfa *n, const int32_t *sources, int32_t n_sources,
                            uint64_t *out_bitmaps, uint32_t flags, rpq_stats *stats) {
    TraceRange tr_("rpq_multi_source");
    return stacked_run(g, n, sources, n_sources, out_bitmaps, flags, stats, "rpq_multi_source", nullptr);
}
