// Served path: rpq_submit / rpq_poll (continuous batching of independent queries).
//
// A scheduler thread owns a multi-query engine (multi.hip). Each admitted
// query occupies a slot with its own state words; every iteration of the loop
//   1. admits queued requests into free slots (bounded by max_slots and the
//      device-memory budget),
//   2. runs ONE level of Alg. 1 for every admitted query in shared launches
//      (select over the combined frontier queue, then edge-balanced push),
//   3. retires the queries whose frontier became empty (one extract launch for
//      all of them), copies their bitmaps out and wakes their pollers.
// New requests therefore join while others are in flight (iteration-level
// scheduling), and one launch carries the work of all of them.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include "api_internal.h"
#include "trace.h"
#include "multi.h"

using namespace rpq;
using Clock = std::chrono::steady_clock;

namespace rpq {

struct Request {
    rpq_ticket id = 0;
    int32_t source = 0;
    int32_t nsym = 0;
    uint32_t smask = 0;
    uint64_t serial = 0;                // the NFA handle's identity
    std::shared_ptr<const rpq_nfa> nfa; // a copy of the NFA (for a stacked group)
    std::vector<uint8_t> qc;            // query constants (build_qconst layout)
    Clock::time_point submitted;
    bool has_deadline = false;          // rpq_submit_deadline: must start by `deadline`
    Clock::time_point deadline;
};

struct Ticket {
    int state = 0;  // 0 queued, 1 running, 2 done, 3 being collected by rpq_poll
    rpq_status status = RPQ_OK;
    std::string error;
    int64_t entry = -1;          // result-pool entry holding the bitmap (done, RPQ_OK)
    std::vector<uint64_t> spill; // or the bitmap in host memory (the pool was full)
    bool empty_result = false;   // no start state: the answer is empty
    rpq_stats stats{};
    bool has_deadline = false;   // a queued request that has not started by `deadline` is dropped
    Clock::time_point deadline;
};

struct SlotInfo {
    rpq_ticket ticket = 0;
    int32_t nsym = 0;
    uint32_t admit_level = 0;
    Clock::time_point submitted;
    bool finished = false;  // frontier empty; waiting for a result-pool entry
    uint32_t levels = 0;
    uint64_t pairs = 0;
    bool dead = false;      // moved to a lane (its reached pairs passed serve_promote_pairs)
    Request req;            // the request, kept for a move to a lane
};

struct ServeState {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> pending;
    size_t pending_deadlines = 0;  // requests in `pending` with a deadline
    Clock::time_point last_submit{};  // arrival of the latest request (guarded by mu)
    std::unordered_map<rpq_ticket, Ticket> tickets;
    std::thread worker;
    bool stop = false;
    bool failed = false;
    std::string fail_msg;
    rpq_ticket next_ticket = 1;
    size_t running = 0;
    // size of recent queries (reached pairs, moving average): while they are
    // large, fewer run at once (the state arrays of many large queries thrash
    // the caches and the TLB; a few already fill the GPU)
    double size_avg = 0.0;
    uint64_t size_n = 0;
    // stacked groups: staging for their answers; grouping is switched off
    // after a failure of the stacked path
    uint64_t *gout = nullptr;
    bool group_off = false;
    // engine (owned by the worker thread after start)
    MultiParams mp{};
    hipStream_t stream = nullptr;
    std::vector<void *> allocs;
    uint8_t *pinned = nullptr;
    size_t pinned_bytes = 0;
    uint32_t slots = 0;
    std::vector<SlotInfo> slot;
    std::vector<uint32_t> free_slots;
    uint32_t level = 0;
    uint32_t chunk_id = 0;
    uint32_t cur_len = 0, prev_len = 0;
    uint8_t *d_stage = nullptr;  // admission upload: records, then query constants (stage_bytes)
    size_t stage_bytes = 0;
    uint32_t *d_hctl = nullptr;  // h_ctl as the device addresses it
    // rpq_poll's copies out of the pool signal completion through a pinned
    // word (h_copy_flag; d_copy_flag as the device addresses it)
    uint32_t *d_copy_done = nullptr;
    uint32_t *d_copy_flag = nullptr;
    volatile uint32_t *h_copy_flag = nullptr;
    uint32_t copy_seq = 0;  // guarded by copy_mu
    // result pool: finished queries' bitmaps stay on the device until polled
    // (entries [0, pool_n)); entries [pool_n, pool_n + slots) stage answers
    // that spill to host memory while every pool entry is held
    uint32_t pool_n = 0;
    std::vector<uint32_t> free_entries;  // guarded by mu
    std::vector<uint32_t> ready;         // finished slots to retire (worker only)
    // lanes: single-query executors (exec_clone) that run the requests of
    // large-query periods side by side, one thread each; lane_q holds the
    // requests handed to them and lanes_busy counts those not finished
    std::vector<rpq_graph *> lanes;
    std::vector<std::thread> lane_threads;
    std::deque<Request> lane_q;
    std::condition_variable cv_lane;
    uint32_t lanes_busy = 0;
    bool lanes_failed = false;  // no lane could be made: run requests in the scheduler thread
    uint32_t *h_one = nullptr;           // pinned word 1: the value a slot's dead flag is set to
    hipStream_t copy_stream = nullptr;   // rpq_poll's copies out of the pool
    std::mutex copy_mu;
    // pinned host staging
    uint32_t *h_fin = nullptr;    // 2 * slots: (slot, pool entry)
    uint8_t *h_ctl = nullptr;     // control block (written by the publish kernel)
    uint8_t *h_stage = nullptr;   // admission upload (stage_bytes)
    int grid = 1024;
};

}  // namespace rpq

static int vbits_for(int32_t V) {
    int b = 1;
    while ((1ll << b) < V) b++;
    return b;
}

static hipError_t salloc(ServeState *ss, void **p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 64);
    if (e == hipSuccess) ss->allocs.push_back(*p);
    return e;
}

// Allocates the engine for `slots` queries. Called by the worker thread.
static rpq_status engine_init(rpq_graph *g, ServeState *ss) {
    const int32_t V = g->V;
    const uint32_t vb = static_cast<uint32_t>(vbits_for(V));
    uint64_t max_by_bits = vb >= 32 ? 1 : (1ull << (32 - vb));
    uint32_t slots = static_cast<uint32_t>(std::min<uint64_t>(static_cast<uint64_t>(g->max_slots), max_by_bits));
    const uint64_t swords = static_cast<uint64_t>(V) + 64;
    // per slot: P and two frontier arrays (4 B/vertex), two queue shares
    // (4 B/vertex), query constants and three result-pool bitmaps
    const uint64_t per_slot = 3 * 4 * swords + 2 * 4 * static_cast<uint64_t>(V) + QC_STRIDE + 24 * g->nwords;
    int64_t budget = g->mem_budget;
    if (budget <= 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(RPQ_EDEVICE, "hipMemGetInfo failed");
        budget = static_cast<int64_t>(fr / 4);
    }
    // the item buffer bounds how many queue entries one select handles (each
    // may yield an item per used symbol); up to 2^26 items, at most an eighth
    // of the budget
    uint64_t item_cap = std::min<uint64_t>(MAX_MULTI_ITEMS - 1, static_cast<uint64_t>(g->rows[OUT] + g->rows[IN]) * 4 + 4096);
    item_cap = std::max<uint64_t>(4096, std::min<uint64_t>(item_cap, static_cast<uint64_t>(budget) / (8 * 20)));
    const uint64_t fixed = item_cap * 20 + (2 * static_cast<uint64_t>(g->E) * slots) / TILE * 4;
    if (static_cast<int64_t>(fixed + per_slot) > budget)
        return fail(RPQ_ENOMEM, "served path: memory budget %lld bytes is below one slot (%llu bytes)",
                    (long long)budget, (unsigned long long)(fixed + per_slot));
    slots = static_cast<uint32_t>(std::min<uint64_t>(slots, (budget - fixed) / per_slot));
    if (slots < 1) slots = 1;
    {
        std::lock_guard<std::mutex> lk(ss->mu);
        ss->slots = slots;
    }
    MultiParams &p = ss->mp;
    p.g = g->gv;
    p.slots = slots;
    p.vbits = vb;
    p.V = V;
    p.swords = swords;
    p.queue_cap = static_cast<uint64_t>(slots) * V;
    p.item_cap = item_cap;
    p.tile_cap = (2 * static_cast<uint64_t>(g->E) * slots) / TILE + 2;
    hipError_t e = hipSuccess;
#define SA(ptr, bytes)                                                                            \
    if ((e = salloc(ss, reinterpret_cast<void **>(&(ptr)), (bytes))) != hipSuccess)               \
        return fail(RPQ_ENOMEM, "served path: hipMalloc %s: %s", #ptr, hipGetErrorString(e));
    uint8_t *qc = nullptr;
    SA(qc, QC_STRIDE * slots);
    p.qconst = qc;
    SA(p.P, 4 * swords * slots);
    SA(p.M[0], 4 * swords * slots);
    SA(p.M[1], 4 * swords * slots);
    SA(p.q[0], 4 * p.queue_cap);
    SA(p.q[1], 4 * p.queue_cap);
    SA(p.ctl, multi_ctl_bytes(slots));
    uint8_t *ctl8 = reinterpret_cast<uint8_t *>(p.ctl);
    p.qlen[0] = reinterpret_cast<uint32_t *>(ctl8 + CTL_QLEN);
    p.qlen[1] = reinterpret_cast<uint32_t *>(ctl8 + CTL_QLEN + CTL_LINE);
    p.status = reinterpret_cast<uint32_t *>(ctl8 + CTL_STATUS);
    p.next_count = reinterpret_cast<uint32_t *>(ctl8 + CTL_NEXT);
    p.pairs = reinterpret_cast<uint64_t *>(ctl8 + multi_pairs_offset(slots));
    SA(p.sel, 64);
    SA(p.it_ebase, 8 * item_cap);
    SA(p.it_beg, 4 * item_cap);
    SA(p.it_mask, 4 * item_cap);
    SA(p.it_slot, 4 * item_cap);
    SA(p.tile_first, 4 * p.tile_cap);
    ss->pool_n = 2 * slots;
    SA(p.out, 8 * g->nwords * (ss->pool_n + slots));
    SA(p.dead, 4 * static_cast<size_t>(slots));
    ss->stage_bytes = ADMIT_TABLE_BYTES + QC_STRIDE * static_cast<size_t>(slots);
    SA(ss->d_stage, ss->stage_bytes);
    SA(ss->d_copy_done, 64);
#undef SA
    const size_t ctl_b = (multi_ctl_bytes(slots) + 63) & ~static_cast<size_t>(63);
    ss->pinned_bytes = ss->stage_bytes + ctl_b + 8 * slots + 256 + 64;
    if ((e = hipHostMalloc(reinterpret_cast<void **>(&ss->pinned), ss->pinned_bytes, hipHostMallocDefault)) != hipSuccess)
        return fail(RPQ_ENOMEM, "served path: hipHostMalloc: %s", hipGetErrorString(e));
    uint8_t *hp = ss->pinned;
    ss->h_stage = hp;
    hp += ss->stage_bytes;
    ss->h_ctl = hp;
    hp += ctl_b;
    ss->h_fin = reinterpret_cast<uint32_t *>(hp);
    hp += 8 * slots;
    ss->h_copy_flag = reinterpret_cast<volatile uint32_t *>(hp);
    *ss->h_copy_flag = 0;
    ss->h_one = reinterpret_cast<uint32_t *>(hp + 256);
    *ss->h_one = 1;
    {
        uint8_t *dp = nullptr;
        if ((e = hipHostGetDevicePointer(reinterpret_cast<void **>(&dp), ss->pinned, 0)) != hipSuccess)
            return hip_fail(e, "hipHostGetDevicePointer");
        ss->d_hctl = reinterpret_cast<uint32_t *>(dp + (ss->h_ctl - ss->pinned));
        ss->d_copy_flag = reinterpret_cast<uint32_t *>(dp + (reinterpret_cast<uint8_t *>(hp) - ss->pinned));
    }
    if ((e = hipStreamCreateWithFlags(&ss->stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreate");
    if ((e = hipStreamCreateWithFlags(&ss->copy_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreate");
    for (uint32_t *a : {p.P, p.M[0], p.M[1]})
        if ((e = launch_fill(a, swords * slots, 0, ss->stream)) != hipSuccess) return hip_fail(e, "fill");
    if ((e = launch_fill(p.ctl, multi_ctl_bytes(slots) / 4, 0, ss->stream)) != hipSuccess) return hip_fail(e, "fill");
    if ((e = launch_fill(p.dead, slots, 0, ss->stream)) != hipSuccess) return hip_fail(e, "fill");
    if ((e = launch_fill(ss->d_copy_done, 16, 0, ss->stream)) != hipSuccess) return hip_fail(e, "fill");
    if ((e = launch_fill(reinterpret_cast<uint32_t *>(p.sel), 4, 0, ss->stream)) != hipSuccess)
        return hip_fail(e, "fill");
    if ((e = hipStreamSynchronize(ss->stream)) != hipSuccess) return hip_fail(e, "sync");
    ss->slot.assign(slots, SlotInfo{});
    for (uint32_t s = slots; s-- > 0;) ss->free_slots.push_back(s);
    {
        std::lock_guard<std::mutex> lk(ss->mu);
        for (uint32_t k = ss->pool_n; k-- > 0;) ss->free_entries.push_back(k);
    }
    return RPQ_OK;
}

#define ST(call)                                                  \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return hip_fail(e_, #call);         \
    } while (0)

static rpq_status retire(rpq_graph *g, ServeState *ss);

// One scheduler iteration with the lock released. Returns a failure status
// for a device error (the engine then stops and fails every ticket).
static rpq_status engine_step(rpq_graph *g, ServeState *ss, std::vector<Request> &admit) {
    TraceRange tr_("served slot level %lld", static_cast<long long>(ss->level));
    MultiParams &p = ss->mp;
    hipStream_t s = ss->stream;
    const uint32_t parity = ss->level & 1;
    // 1. admission: one upload of the requests' records and query constants;
    //    the admit kernel moves the constants into the slots and sets the
    //    start pairs
    if (!admit.empty()) {
        uint32_t k = 0;
        uint32_t *table = reinterpret_cast<uint32_t *>(ss->h_stage);
        size_t off = ADMIT_TABLE_BYTES;
        for (Request &r : admit) {
            const uint32_t sl = ss->free_slots.back();
            ss->free_slots.pop_back();
            ss->slot[sl] = SlotInfo{r.id, r.nsym, ss->level, r.submitted};
            // admit.size() <= free slots <= slots, each block <= QC_STRIDE: it fits
            memcpy(ss->h_stage + off, r.qc.data(), r.qc.size());
            table[4 * k] = sl;
            table[4 * k + 1] = static_cast<uint32_t>(r.source);
            table[4 * k + 2] = static_cast<uint32_t>(off);
            table[4 * k + 3] = static_cast<uint32_t>(r.qc.size());
            off += (r.qc.size() + 15) & ~static_cast<size_t>(15);
            k++;
            ss->slot[sl].req = std::move(r);
        }
        ST(hipMemcpyAsync(ss->d_stage, ss->h_stage, off, hipMemcpyHostToDevice, s));
        ST(multi_admit(p, parity, k, ss->d_stage, s));
        ss->cur_len += k;  // every admitted request has a start state (checked at submit)
    }
    if (ss->cur_len == 0) return retire(g, ss);
    // 2. one level for every admitted query, in chunks bounded by the item buffer
    int32_t maxsym = 1;
    for (uint32_t sl = 0; sl < ss->slots; sl++)
        if (ss->slot[sl].ticket) maxsym = std::max(maxsym, ss->slot[sl].nsym);
    const uint32_t chunk = static_cast<uint32_t>(std::max<uint64_t>(1, p.item_cap / static_cast<uint64_t>(maxsym)));
    for (uint32_t lo = 0; lo < ss->cur_len; lo += chunk) {
        const uint32_t hi = std::min(ss->cur_len, lo + chunk);
        ST(multi_select(p, parity, lo, hi, ss->prev_len, lo == 0, ss->chunk_id, ss->grid, s));
        ST(multi_push(p, parity, ss->chunk_id, ss->grid, s));
        ss->chunk_id++;
    }
    ST(multi_publish(p, ss->d_hctl, static_cast<uint32_t>(multi_ctl_bytes(ss->slots) / 4), s));
    ST(hipStreamSynchronize(s));
    const uint32_t h_status = *reinterpret_cast<const uint32_t *>(ss->h_ctl + CTL_STATUS);
    const uint32_t *h_cnt = reinterpret_cast<const uint32_t *>(ss->h_ctl + CTL_NEXT);
    const uint64_t *h_pairs = reinterpret_cast<const uint64_t *>(ss->h_ctl + multi_pairs_offset(ss->slots));
    if (h_status) return fail(RPQ_EDEVICE, "served path: internal invariant violated %u times", h_status);
    const uint32_t next_len = *reinterpret_cast<const uint32_t *>(ss->h_ctl + CTL_QLEN + (parity ^ 1) * CTL_LINE);
    // 3. queries whose next frontier is empty are finished; a query whose
    //    reached pairs passed serve_promote_pairs moves to a lane: its slot's
    //    candidates are dropped from the next select on (the flag goes up
    //    on this stream, ahead of the next level), its frontier ends there,
    //    and retire() hands the request to the lanes instead of answering
    const uint64_t promote = (g->serve_promote_pairs > 0 && !ss->lanes.empty())
                                 ? static_cast<uint64_t>(g->serve_promote_pairs) : 0;
    for (uint32_t sl = 0; sl < ss->slots; sl++) {
        SlotInfo &si = ss->slot[sl];
        if (si.ticket && !si.finished && h_cnt[sl] == 0) {
            si.finished = true;
            si.levels = ss->level - si.admit_level + 1;
            si.pairs = h_pairs[sl * PAIRS_STRIDE];
            ss->ready.push_back(sl);
        } else if (si.ticket && !si.finished && !si.dead && promote && h_pairs[sl * PAIRS_STRIDE] > promote) {
            si.dead = true;
            ST(hipMemcpyAsync(p.dead + sl, ss->h_one, 4, hipMemcpyHostToDevice, s));
        }
    }
    ss->prev_len = ss->cur_len;
    ss->cur_len = next_len;
    ss->level++;
    return retire(g, ss);
}

// Moves finished queries' answers into result-pool entries (one extract
// launch for all of them) and frees their slots. When every pool entry is
// held by an answer nobody has polled yet, the answer is copied to host
// memory instead, so no poll order can stall the scheduler.
static rpq_status retire(rpq_graph *g, ServeState *ss) {
    if (ss->ready.empty()) return RPQ_OK;
    MultiParams &p = ss->mp;
    hipStream_t s = ss->stream;
    const uint32_t nfin = static_cast<uint32_t>(ss->ready.size());  // <= slots
    uint32_t nspill = 0;
    {
        std::lock_guard<std::mutex> lk(ss->mu);
        for (uint32_t f = 0; f < nfin; f++) {
            ss->h_fin[2 * f] = ss->ready[f];
            if (ss->slot[ss->ready[f]].dead) {
                // extracted only to clear the slot: a staging entry, not copied out
                ss->h_fin[2 * f + 1] = ss->pool_n + nspill++;
            } else if (!ss->free_entries.empty()) {
                ss->h_fin[2 * f + 1] = ss->free_entries.back();
                ss->free_entries.pop_back();
            } else {
                ss->h_fin[2 * f + 1] = ss->pool_n + nspill++;
            }
        }
    }
    {
        FinList fl;
        fl.n = nfin;
        memcpy(fl.e, ss->h_fin, 8 * static_cast<size_t>(nfin));
        ST(multi_extract(p, fl, static_cast<uint64_t>(g->nwords), s));
    }
    ST(hipStreamSynchronize(s));
    std::vector<std::vector<uint64_t>> spilled(nspill);
    for (uint32_t f = 0, k = 0; f < nfin; f++) {
        const uint32_t entry = ss->h_fin[2 * f + 1];
        if (entry < ss->pool_n) continue;
        if (ss->slot[ss->h_fin[2 * f]].dead) {
            k++;
            continue;
        }
        spilled[k].resize(static_cast<size_t>(g->nwords));
        ST(hipMemcpy(spilled[k].data(), p.out + static_cast<size_t>(entry) * g->nwords, 8 * static_cast<size_t>(g->nwords),
                     hipMemcpyDeviceToHost));
        k++;
    }
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> lk(ss->mu);
    for (uint32_t f = 0, k = 0; f < nfin; f++) {
        const uint32_t sl = ss->h_fin[2 * f];
        const uint32_t entry = ss->h_fin[2 * f + 1];
        const bool spill = entry >= ss->pool_n;
        SlotInfo &si = ss->slot[sl];
        auto it = ss->tickets.find(si.ticket);
        if (si.dead) {
            // the request runs again on a lane from its start (answered there)
            if (spill) k++;
            ss->lane_q.push_front(std::move(si.req));
            ss->lanes_busy++;
            ss->cv_lane.notify_one();
            si = SlotInfo{};
            ss->free_slots.push_back(sl);
            continue;
        }
        if (it != ss->tickets.end()) {
            Ticket &t = it->second;
            if (spill) t.spill.swap(spilled[k]);
            else t.entry = entry;
            t.stats = rpq_stats{};
            t.stats.levels = static_cast<int32_t>(si.levels);
            t.stats.push_levels = t.stats.levels;
            t.stats.visited_pairs = static_cast<int64_t>(si.pairs);
            t.stats.latency_ms = std::chrono::duration<double, std::milli>(now - si.submitted).count();
            t.stats.batch = static_cast<int32_t>(ss->slots - ss->free_slots.size());
            t.status = RPQ_OK;
            t.state = 2;
        } else if (!spill) {
            ss->free_entries.push_back(entry);
        }
        if (spill) k++;
        ss->size_avg = ss->size_n == 0 ? static_cast<double>(si.pairs)
                                       : 0.8 * ss->size_avg + 0.2 * static_cast<double>(si.pairs);
        ss->size_n++;
        si = SlotInfo{};
        ss->free_slots.push_back(sl);
        ss->running--;
    }
    ss->ready.clear();
    ss->cv_done.notify_all();
    return RPQ_OK;
}

// Requests that share one NFA and wait together run as one stacked
// multi-source traversal (every source one bit of a stacked row: the same
// answers, one pass over the graph for all of them) into a staging buffer;
// each answer then moves to a result-pool entry or, when none is free, to
// host memory. Called by the worker thread without ss->mu held.
static rpq_status run_group(rpq_graph *g, ServeState *ss, std::vector<Request> &grp) {
    TraceRange tr_("served stacked group of %lld", static_cast<long long>(grp.size()));
    const int32_t B = static_cast<int32_t>(grp.size());
    const size_t nw = static_cast<size_t>(g->nwords);
    if (!ss->gout) {
        const size_t words = static_cast<size_t>(std::min<int32_t>(g->max_batch, MAX_BATCH)) * nw;
        ST(salloc(ss, reinterpret_cast<void **>(&ss->gout), 8 * words));
    }
    std::vector<int32_t> src(static_cast<size_t>(B));
    for (int32_t i = 0; i < B; i++) src[i] = grp[i].source;
    rpq_stats stt{};
    rpq_status st = rpq_multi_source(g, grp[0].nfa.get(), src.data(), B, ss->gout, RPQ_OUT_DEVICE, &stt);
    if (st != RPQ_OK) return st;
    std::vector<uint32_t> entry(static_cast<size_t>(B), ~0u);
    {
        std::lock_guard<std::mutex> lk(ss->mu);
        for (int32_t i = 0; i < B && !ss->free_entries.empty(); i++) {
            entry[i] = ss->free_entries.back();
            ss->free_entries.pop_back();
        }
    }
    std::vector<std::vector<uint64_t>> spill(static_cast<size_t>(B));
    for (int32_t i = 0; i < B; i++) {
        const uint64_t *from = ss->gout + static_cast<size_t>(i) * nw;
        if (entry[i] != ~0u) {
            ST(hipMemcpyAsync(ss->mp.out + static_cast<size_t>(entry[i]) * nw, from, 8 * nw, hipMemcpyDeviceToDevice,
                              ss->stream));
        } else {
            spill[i].resize(nw);
            ST(hipMemcpyAsync(spill[i].data(), from, 8 * nw, hipMemcpyDeviceToHost, ss->stream));
        }
    }
    ST(hipStreamSynchronize(ss->stream));
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> lk(ss->mu);
    for (int32_t i = 0; i < B; i++) {
        auto it = ss->tickets.find(grp[i].id);
        if (it != ss->tickets.end()) {
            Ticket &t = it->second;
            if (entry[i] != ~0u) t.entry = entry[i];
            else t.spill.swap(spill[i]);
            // a stacked group's statistics: its level count and total pairs
            t.stats = rpq_stats{};
            t.stats.levels = stt.levels;
            t.stats.push_levels = stt.push_levels;
            t.stats.pull_levels = stt.pull_levels;
            t.stats.visited_pairs = stt.visited_pairs;
            t.stats.latency_ms = std::chrono::duration<double, std::milli>(now - grp[i].submitted).count();
            t.stats.batch = B;
            t.status = RPQ_OK;
            t.state = 2;
        } else if (entry[i] != ~0u) {
            ss->free_entries.push_back(entry[i]);
        }
        ss->running--;
    }
    ss->cv_done.notify_all();
    return RPQ_OK;
}

// A request run alone by the single-query persistent kernel (while recent
// queries are large: for them it is the most efficient path per edge), its
// answer written straight into a result-pool entry or, when none is free,
// into host memory. Called by the worker thread without ss->mu held.
static void run_one(rpq_graph *g, ServeState *ss, Request &r) {
    TraceRange tr_("served query %lld", static_cast<long long>(r.id));
    const size_t nw = static_cast<size_t>(g->nwords);
    uint32_t entry = ~0u;
    {
        std::lock_guard<std::mutex> lk(ss->mu);
        if (!ss->free_entries.empty()) {
            entry = ss->free_entries.back();
            ss->free_entries.pop_back();
        }
    }
    std::vector<uint64_t> spill;
    rpq_stats st{};
    rpq_status rs;
    if (entry != ~0u) {
        rs = rpq_single_source(g, r.nfa.get(), r.source, ss->mp.out + static_cast<size_t>(entry) * nw, RPQ_OUT_DEVICE,
                               &st);
    } else {
        spill.resize(nw);
        rs = rpq_single_source(g, r.nfa.get(), r.source, spill.data(), 0u, &st);
    }
    const std::string err = rs == RPQ_OK ? std::string() : std::string(rpq_last_error());
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> lk(ss->mu);
    auto it = ss->tickets.find(r.id);
    if (it != ss->tickets.end()) {
        Ticket &t = it->second;
        t.stats = rpq_stats{};
        if (rs == RPQ_OK) {
            if (entry != ~0u) t.entry = entry;
            else t.spill.swap(spill);
            t.stats.levels = st.levels;
            t.stats.push_levels = st.push_levels;
            t.stats.pull_levels = st.pull_levels;
            t.stats.visited_pairs = st.visited_pairs;
            t.stats.batch = 1;
            t.stats.device_ms = st.device_ms;  // the query ran alone in its own launch
            t.stats.latency_ms = std::chrono::duration<double, std::milli>(now - r.submitted).count();
        } else {
            t.error = err;
            if (entry != ~0u) ss->free_entries.push_back(entry);
        }
        t.status = rs;
        t.state = 2;
    } else if (entry != ~0u) {
        ss->free_entries.push_back(entry);
    }
    if (rs == RPQ_OK) {
        ss->size_avg = ss->size_n == 0 ? static_cast<double>(st.visited_pairs)
                                       : 0.8 * ss->size_avg + 0.2 * static_cast<double>(st.visited_pairs);
        ss->size_n++;
    }
    ss->running--;
    ss->cv_done.notify_all();
}

// Drops the queued requests whose deadline has passed: their tickets finish
// with RPQ_ETIMEDOUT. Called with ss->mu held.
static void expire_pending(ServeState *ss, Clock::time_point now) {
    if (ss->pending_deadlines == 0) return;
    bool any = false;
    for (auto it = ss->pending.begin(); it != ss->pending.end();) {
        if (!it->has_deadline || it->deadline > now) {
            ++it;
            continue;
        }
        auto t = ss->tickets.find(it->id);
        if (t != ss->tickets.end()) {
            t->second.state = 2;
            t->second.status = RPQ_ETIMEDOUT;
            t->second.error = "served request not started within its deadline";
        }
        ss->pending_deadlines--;
        ss->running--;
        it = ss->pending.erase(it);
        any = true;
    }
    if (any) ss->cv_done.notify_all();
}

// Takes the first queued request (its deadline no longer counts).
static Request take_front(ServeState *ss) {
    Request r = std::move(ss->pending.front());
    ss->pending.pop_front();
    if (r.has_deadline) ss->pending_deadlines--;
    auto t = ss->tickets.find(r.id);
    if (t != ss->tickets.end()) {
        t->second.state = 1;
        t->second.has_deadline = false;
    }
    return r;
}

// A lane's thread: runs the requests handed to it through its own
// single-query executor until the served path stops.
static void lane_main(rpq_graph *g, ServeState *ss, rpq_graph *lane) {
    (void)hipSetDevice(g->device);
    while (true) {
        Request r;
        {
            std::unique_lock<std::mutex> lk(ss->mu);
            ss->cv_lane.wait(lk, [&] { return ss->stop || !ss->lane_q.empty(); });
            if (ss->lane_q.empty()) return;
            r = std::move(ss->lane_q.front());
            ss->lane_q.pop_front();
        }
        {
            std::lock_guard<std::recursive_mutex> glk(g->mu);  // options are set under it
            exec_sync_options(lane, g);
            if (ss->lanes.size() > 2 && g->pgrid[1] > 0) {
                // more lanes than two full grids fit: each gets its share
                const int share = std::max(1, static_cast<int>(2 * g->pgrid[1] / ss->lanes.size()));
                lane->plain_grid = lane->plain_grid ? std::min(lane->plain_grid, share) : share;
            }
        }
        run_one(lane, ss, r);
        {
            std::lock_guard<std::mutex> lk(ss->mu);
            ss->lanes_busy--;
        }
        ss->cv_work.notify_all();
    }
}

// Makes the lanes at their first use (in the scheduler thread). Returns the
// number of lanes; 0 when none could be made (their memory), after which
// large requests run in the scheduler thread one at a time.
static size_t lanes_ready(rpq_graph *g, ServeState *ss) {
    if (!ss->lanes.empty() || ss->lanes_failed) return ss->lanes.size();
    const int32_t want = std::max<int32_t>(0, g->serve_lanes);
    std::vector<rpq_graph *> made;
    for (int32_t k = 0; k < want; k++) {
        rpq_graph *c = nullptr;
        if (exec_clone(g, &c) != RPQ_OK) break;
        made.push_back(c);
    }
    std::lock_guard<std::mutex> lk(ss->mu);
    if (made.empty()) {
        ss->lanes_failed = true;
        return 0;
    }
    ss->lanes = made;
    for (rpq_graph *c : ss->lanes) ss->lane_threads.emplace_back(lane_main, g, ss, c);
    return ss->lanes.size();
}

static void fail_all(ServeState *ss, rpq_status st, const std::string &msg) {
    std::lock_guard<std::mutex> lk(ss->mu);
    ss->failed = true;
    ss->fail_msg = msg;
    for (auto &kv : ss->tickets)
        if (kv.second.state != 2) {
            kv.second.state = 2;
            kv.second.status = st;
            kv.second.error = msg;
        }
    ss->pending.clear();
    ss->pending_deadlines = 0;
    ss->running = 0;
    ss->cv_done.notify_all();
}

static void worker_main(rpq_graph *g, ServeState *ss) {
    if (hipSetDevice(g->device) != hipSuccess) {
        fail_all(ss, RPQ_EDEVICE, "served path: hipSetDevice failed");
        return;
    }
    rpq_status st = engine_init(g, ss);
    if (st != RPQ_OK) {
        fail_all(ss, st, rpq_last_error());
        return;
    }
    std::vector<Request> admit, grp, one;
    bool make_lanes = false;
    // with promotion, the lanes exist from the start: large queries move
    // there from their slots while the slots go on with the rest
    if (g->serve_promote_pairs > 0 && g->serve_lanes > 0) lanes_ready(g, ss);
    while (true) {
        admit.clear();
        grp.clear();
        one.clear();
        if (make_lanes) {
            lanes_ready(g, ss);  // outside ss->mu: it allocates their state
            make_lanes = false;
        }
        {
            std::unique_lock<std::mutex> lk(ss->mu);
            expire_pending(ss, Clock::now());
            // a stacked group: at least serve_stack_min waiting requests of one NFA
            const size_t smin = ss->group_off ? 0 : static_cast<size_t>(std::max<int32_t>(g->serve_stack_min, 0));
            auto group_serial = [&]() -> uint64_t {
                if (smin == 0 || ss->pending.size() < smin) return 0;
                std::unordered_map<uint64_t, size_t> cnt;
                for (const Request &r : ss->pending)
                    if (++cnt[r.serial] >= smin) return r.serial;
                return 0;
            };
            // a burst of one NFA's requests (half a group or more waiting,
            // the last one recent) is held back from the slots for a short
            // while, and a group short of max_batch waits as long for more
            // of its requests, so that the burst gathers into one group
            const auto gwait = std::chrono::microseconds(smin ? std::max<int64_t>(g->serve_group_wait_us, 0) : 0);
            const size_t maxb = static_cast<size_t>(std::min<int32_t>(g->max_batch, MAX_BATCH));
            // (a group also starts once its oldest request has waited 25
            // windows, so a steady trickle of one NFA's requests is not held
            // until max_batch of them have come)
            auto group_ready = [&]() -> uint64_t {
                const uint64_t gsr = group_serial();
                const Clock::time_point now = Clock::now();
                if (!gsr || gwait.count() == 0 || now - ss->last_submit >= gwait) return gsr;
                size_t c = 0;
                Clock::time_point oldest = now;
                for (const Request &r : ss->pending)
                    if (r.serial == gsr) {
                        c++;
                        oldest = std::min(oldest, r.submitted);
                    }
                return c >= maxb || now - oldest >= 25 * gwait ? gsr : 0;
            };
            const size_t hmin = std::max<size_t>(2, smin / 2);
            auto holding = [&]() -> bool {
                if (gwait.count() == 0 || ss->pending.size() < hmin || Clock::now() - ss->last_submit >= gwait)
                    return false;
                std::unordered_map<uint64_t, size_t> cnt;
                for (const Request &r : ss->pending)
                    if (++cnt[r.serial] >= hmin) return true;
                return false;
            };
            // concurrency: every slot, or large_query_slots while recent
            // queries are large; with large_query_slots 0, large-query
            // periods run one request at a time through the single-query
            // kernel once the slots have drained
            const bool promoting = g->serve_promote_pairs > 0 && !ss->lanes.empty();
            const bool large = !promoting && ss->size_n && ss->size_avg > static_cast<double>(g->large_pairs);
            size_t cap = ss->slots;
            if (large) cap = std::min<size_t>(cap, static_cast<size_t>(g->large_slots));
            auto active = [&] { return static_cast<size_t>(ss->slots) - ss->free_slots.size(); };
            const bool single = large && g->large_slots == 0;
            // the lanes that run such requests (none: they run in this thread)
            const size_t nl = ss->lanes.size();
            // work: a level to run, a request and a free slot, a group, or a
            // request to run through the single-query kernel
            auto ready = [&] {
                return ss->stop || ss->cur_len > 0 ||
                       (!ss->pending.empty() && !ss->free_slots.empty() && active() < cap && !holding()) ||
                       group_ready() != 0 ||
                       (single && !ss->pending.empty() && active() == 0 && (nl == 0 || ss->lanes_busy < nl));
            };
            while (!ready()) {
                // a held burst is looked at again when its window closes
                const Clock::time_point until = ss->last_submit + gwait;
                if (gwait.count() > 0 && !ss->pending.empty() && Clock::now() < until)
                    ss->cv_work.wait_until(lk, until);
                else
                    ss->cv_work.wait(lk);
            }
            if (ss->stop && ss->pending.empty() && ss->cur_len == 0) break;
            const uint64_t gs = ss->stop ? 0 : group_ready();
            if (!gs && single && ss->cur_len == 0 && active() == 0 && !ss->pending.empty()) {
                if (nl == 0 && g->serve_lanes > 0 && !ss->lanes_failed) {
                    make_lanes = true;
                    continue;
                }
                if (nl == 0) {
                    one.push_back(take_front(ss));
                } else {
                    // hand requests to the free lanes
                    while (!ss->pending.empty() && ss->lanes_busy < nl) {
                        ss->lane_q.push_back(take_front(ss));
                        ss->lanes_busy++;
                    }
                    ss->cv_lane.notify_all();
                    continue;
                }
            } else if (gs) {
                for (auto it = ss->pending.begin(); it != ss->pending.end() && grp.size() < maxb;) {
                    if (it->serial != gs) {
                        ++it;
                        continue;
                    }
                    grp.push_back(std::move(*it));
                    it = ss->pending.erase(it);
                    if (grp.back().has_deadline) ss->pending_deadlines--;
                    auto t = ss->tickets.find(grp.back().id);
                    if (t != ss->tickets.end()) {
                        t->second.state = 1;
                        t->second.has_deadline = false;
                    }
                }
            } else if (!holding()) {
                while (!ss->pending.empty() && admit.size() < ss->free_slots.size() &&
                       active() + admit.size() < cap)
                    admit.push_back(take_front(ss));
            }
        }
        if (!one.empty()) {
            run_one(g, ss, one[0]);
            continue;
        }
        if (!grp.empty()) {
            if (run_group(g, ss, grp) != RPQ_OK) {
                // the stacked path failed (for instance no memory for its
                // state): these requests go back to the queue for the slots,
                // and grouping stays off
                std::lock_guard<std::mutex> lk(ss->mu);
                for (size_t i = grp.size(); i-- > 0;) {
                    auto t = ss->tickets.find(grp[i].id);
                    if (t != ss->tickets.end()) t->second.state = 0;
                    grp[i].has_deadline = false;  // it had started
                    ss->pending.push_front(std::move(grp[i]));
                }
                ss->group_off = true;
            }
            continue;
        }
        st = engine_step(g, ss, admit);
        if (st != RPQ_OK) {
            fail_all(ss, st, rpq_last_error());
            return;
        }
    }
}

static ServeState *serve_get(rpq_graph *g) {
    std::lock_guard<std::mutex> lk(g->serve_mu);
    ServeState *ss = g->serve.load();
    if (!ss) {
        ss = new ServeState();
        ss->worker = std::thread(worker_main, g, ss);
        g->serve.store(ss);
    }
    return ss;
}

void rpq::serve_shutdown(rpq_graph *g) {
    ServeState *ss = g->serve;
    if (!ss) return;
    {
        std::lock_guard<std::mutex> lk(ss->mu);
        ss->stop = true;
        ss->pending.clear();
        ss->pending_deadlines = 0;
    }
    ss->cv_work.notify_all();
    if (ss->worker.joinable()) ss->worker.join();
    {
        std::lock_guard<std::mutex> lk(ss->mu);
        ss->lane_q.clear();
    }
    ss->cv_lane.notify_all();
    for (std::thread &t : ss->lane_threads)
        if (t.joinable()) t.join();
    for (rpq_graph *c : ss->lanes) exec_free(c);
    if (ss->stream) (void)hipStreamDestroy(ss->stream);
    if (ss->copy_stream) (void)hipStreamDestroy(ss->copy_stream);
    if (ss->pinned) (void)hipHostFree(ss->pinned);
    for (void *p : ss->allocs) (void)hipFree(p);
    delete ss;
    g->serve = nullptr;
}

int64_t rpq::serve_slots(rpq_graph *g) {
    ServeState *ss = g->serve;
    if (!ss) return 0;
    std::lock_guard<std::mutex> lk(ss->mu);
    return static_cast<int64_t>(ss->slots);
}

int64_t rpq::serve_lane_count(rpq_graph *g) {
    ServeState *ss = g->serve;
    if (!ss) return 0;
    std::lock_guard<std::mutex> lk(ss->mu);
    return static_cast<int64_t>(ss->lanes.size());
}

bool rpq::serve_pending(rpq_graph *g) {
    ServeState *ss = g->serve;
    if (!ss) return false;
    std::lock_guard<std::mutex> lk(ss->mu);
    for (auto &kv : ss->tickets)
        if (kv.second.state != 2) return true;
    return false;
}


static rpq_status submit(rpq_graph *g, const rpq_nfa *n, int32_t source, int64_t deadline_us, rpq_ticket *out);

rpq_status rpq_submit(rpq_graph *g, const rpq_nfa *n, int32_t source, rpq_ticket *out) {
    return submit(g, n, source, 0, out);
}

rpq_status rpq_submit_deadline(rpq_graph *g, const rpq_nfa *n, int32_t source, int64_t deadline_us,
                               rpq_ticket *out) {
    return submit(g, n, source, deadline_us, out);
}

static rpq_status submit(rpq_graph *g, const rpq_nfa *n, int32_t source, int64_t deadline_us, rpq_ticket *out) {
    if (!g || !n || !out) return fail(RPQ_EINVAL, "rpq_submit: NULL argument");
    if (source < 0 || source >= g->V) return fail(RPQ_EINVAL, "rpq_submit: source %d outside [0, %d)", source, g->V);
    Request r;
    r.source = source;
    r.smask = n->smask;
    r.serial = n->serial;
    r.nfa = std::make_shared<const rpq_nfa>(*n);
    const size_t sz = build_qconst(g, n, 1u, 0u, r.qc, &r.nsym);
    if (r.nsym > MAX_SYMS || sz > QC_STRIDE)
        return fail(RPQ_EINVAL, "rpq_submit: query uses %d symbols; the limit is %d", r.nsym, MAX_SYMS);
    r.submitted = Clock::now();
    if (deadline_us > 0) {
        r.has_deadline = true;
        r.deadline = r.submitted + std::chrono::microseconds(deadline_us);
    }
    // no g->mu here: the scheduler holds it while it runs a query through
    // the single-query or stacked path, and a submit must not wait for that
    // (requests queue up while one runs, and can then run as a group)
    ServeState *ss = serve_get(g);
    std::lock_guard<std::mutex> lk(ss->mu);
    if (ss->failed) return fail(RPQ_EDEVICE, "served path failed earlier: %s", ss->fail_msg.c_str());
    const rpq_ticket id = ss->next_ticket++;
    r.id = id;
    Ticket &t = ss->tickets[id];
    if (r.smask == 0) {  // no start state: the answer is empty, nothing to run
        t.state = 2;
        t.empty_result = true;
        t.stats.batch = 1;
    } else {
        t.has_deadline = r.has_deadline;
        t.deadline = r.deadline;
        if (r.has_deadline) ss->pending_deadlines++;
        ss->last_submit = r.submitted;
        ss->pending.push_back(std::move(r));
        ss->running++;
    }
    *out = id;
    ss->cv_work.notify_one();
    return RPQ_OK;
}

rpq_status rpq_poll(rpq_graph *g, rpq_ticket t, uint64_t *out_bitmap, uint32_t flags, rpq_stats *stats,
                    int64_t timeout_us) {
    if (!g || !out_bitmap) return fail(RPQ_EINVAL, "rpq_poll: NULL argument");
    ServeState *ss = g->serve;
    if (!ss) return fail(RPQ_ENOTFOUND, "rpq_poll: unknown ticket %llu", (unsigned long long)t);
    const bool dev = (flags & RPQ_OUT_DEVICE) != 0;
    const size_t bytes = 8 * static_cast<size_t>(g->nwords);
    int64_t entry = -1;
    bool empty = false;
    std::vector<uint64_t> spill;
    rpq_stats tstats{};
    {
        std::unique_lock<std::mutex> lk(ss->mu);
        auto it = ss->tickets.find(t);
        if (it == ss->tickets.end() || it->second.state == 3)
            return fail(RPQ_ENOTFOUND, "rpq_poll: unknown ticket %llu", (unsigned long long)t);
        Ticket &tk = it->second;  // the element stays in place while others are added
        auto done = [&] { return tk.state == 2; };
        const Clock::time_point now = Clock::now();
        const bool bounded = timeout_us >= 0;
        const Clock::time_point until = now + std::chrono::microseconds(bounded ? timeout_us : 0);
        while (!done()) {
            // a queued request whose deadline has passed finishes here
            if (tk.state == 0 && tk.has_deadline && Clock::now() >= tk.deadline) {
                expire_pending(ss, Clock::now());
                continue;
            }
            if (timeout_us == 0) return RPQ_PENDING;
            Clock::time_point wake = bounded ? until : Clock::time_point::max();
            if (tk.state == 0 && tk.has_deadline && tk.deadline < wake) wake = tk.deadline;
            if (wake == Clock::time_point::max()) ss->cv_done.wait(lk);
            else ss->cv_done.wait_until(lk, wake);
            if (!done() && bounded && Clock::now() >= until && !(tk.state == 0 && tk.has_deadline &&
                                                                Clock::now() >= tk.deadline))
                return fail(RPQ_ETIMEDOUT, "rpq_poll: ticket %llu not finished within %lld us", (unsigned long long)t,
                            (long long)timeout_us);
        }
        if (tk.status != RPQ_OK) {
            const rpq_status st = tk.status;
            fail(st, "%s", tk.error.c_str());
            ss->tickets.erase(t);
            return st;
        }
        tk.state = 3;  // this call collects it
        entry = tk.entry;
        empty = tk.empty_result;
        spill.swap(tk.spill);
        tstats = tk.stats;
    }
    // copy the answer out of the result pool (outside the scheduler's lock)
    hipError_t e = hipSuccess;
    if (empty) {
        if (dev) e = hipMemset(out_bitmap, 0, bytes);
        else memset(out_bitmap, 0, bytes);
    } else if (entry < 0) {
        if (dev) e = hipMemcpy(out_bitmap, spill.data(), bytes, hipMemcpyHostToDevice);
        else memcpy(out_bitmap, spill.data(), bytes);
    } else if (dev) {
        // a copy kernel that stores a sequence number into pinned memory once
        // the copy is visible everywhere: the host polls that word for up to
        // 200 us (a stream synchronisation wakes up tens of microseconds
        // late), then waits on the stream
        std::lock_guard<std::mutex> ck(ss->copy_mu);
        const uint32_t seq = ++ss->copy_seq;
        e = copy_signal(ss->mp.out + static_cast<size_t>(entry) * g->nwords, out_bitmap,
                        static_cast<uint64_t>(g->nwords), ss->d_copy_done, ss->d_copy_flag, seq, ss->copy_stream);
        if (e == hipSuccess) {
            const Clock::time_point t0 = Clock::now();
            bool seen = false;
            while (!(seen = (*ss->h_copy_flag == seq)) && Clock::now() - t0 < std::chrono::microseconds(200)) {
            }
            if (!seen) e = hipStreamSynchronize(ss->copy_stream);
        }
    } else {
        std::lock_guard<std::mutex> ck(ss->copy_mu);
        e = hipMemcpyAsync(out_bitmap, ss->mp.out + static_cast<size_t>(entry) * g->nwords, bytes,
                           hipMemcpyDeviceToHost, ss->copy_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ss->copy_stream);
    }
    {
        std::lock_guard<std::mutex> lk(ss->mu);
        if (entry >= 0) ss->free_entries.push_back(static_cast<uint32_t>(entry));
        ss->tickets.erase(t);
    }
    ss->cv_work.notify_one();
    if (e != hipSuccess) return hip_fail(e, "rpq_poll: copying the answer");
    if (stats) {
        rpq_stats in = *stats;
        *stats = tstats;
        stats->level_counts = in.level_counts;
        stats->level_cap = in.level_cap;
        stats->level_us = in.level_us;
        stats->level_frontier = in.level_frontier;
        stats->level_edges = in.level_edges;
        stats->level_select_us = in.level_select_us;
    }
    return RPQ_OK;
}
