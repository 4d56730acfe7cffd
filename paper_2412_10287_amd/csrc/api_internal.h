// Host-side handle structures of librpq.
#pragma once

#include <atomic>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/rpq.h"
#include "graph_build.h"
#include "rpq_internal.h"

// Device bytes per graph handle for cached single-query constants (at least
// 50 queries of the largest kind, thousands of typical ones).
constexpr size_t QARENA_BYTES = size_t(4) << 20;

namespace rpq {

constexpr int64_t MAX_EDGES = (1ll << 31) - (1ll << 16);  // distinct edges per direction
constexpr int32_t MAX_BATCH = 1024;
constexpr int32_t MAX_SLOTS = 256;
constexpr int32_t MAX_LANES = 8;

struct Trans {
    int32_t sym, from, to;
};

struct ServeState;  // serve.cpp
struct BatchState;  // batch.cpp

}  // namespace rpq

struct rpq_nfa {
    int32_t Q = 0, NL = 0;
    uint32_t smask = 0, fmask = 0;
    uint64_t serial = 0;
    std::vector<rpq::Trans> trans;
};

struct rpq_graph {
    int32_t V = 0, L = 0;
    int64_t E = 0;
    int device = 0;
    rpq::GraphView gv{};
    rpq::StateView sv{};
    std::vector<int64_t> label_edges;
    std::vector<int64_t> label_rows[2];  // rows per (direction, label)
    int64_t rows[2] = {0, 0};
    std::vector<uint64_t> rbase;  // [direction * L + label] first rowptr entry
    std::vector<void *> allocs;
    int64_t device_bytes = 0;
    int64_t nwords = 0;
    uint64_t *dev_out = nullptr;
    int32_t *dev_dist = nullptr;    // V lengths for rpq_single_source_lengths with host output (lazy)
    int32_t *dev_srcset = nullptr;  // a start set's distinct vertices for rpq_source_set (lazy, V entries)
    int32_t *pin_srcset = nullptr;  // pinned staging of the same (lazy, V entries)
    uint8_t *qconst_dev = nullptr;
    size_t qconst_cap = 0;
    uint8_t *pinned = nullptr;
    size_t pinned_cap = 0;
    uint32_t *hstat = nullptr;      // pinned status words the single-query kernel writes (StateView::hstat)
    uint32_t *hstat_dev = nullptr;  // the same memory as the device addresses it
    uint32_t hserial = 0;           // serial of the last single-query launch
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t user_stream = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // RPQ_GRAPH_LEVELS: device copy of the query's Params, level control
    // words, the captured level graphs per state-word width (and their grid),
    // and the stream they are captured on (all made at first use)
    rpq::Params *pdev = nullptr;
    uint32_t *gctl = nullptr;
    hipGraphExec_t lgraph[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int lgraph_grid[5] = {0, 0, 0, 0, 0};
    hipStream_t cap_stream = nullptr;
    int pgrid[5] = {0, 0, 0, 0, 0};
    bool dirty = false;
    // persistent-launch barriers, used in turn: each launch zeroes the other
    rpq::GridBarrier *bars[2] = {nullptr, nullptr};
    int bar_idx = 0;
    bool bars_dirty = true;  // zero both before the next launch (first use, or after an aborted launch)
    // options
    double pull_alpha = 0.0;  // push only until tuned (see rpq_set_option)
    double pull_beta = 24.0;
    double stack_alpha = 0.0;  // the same thresholds for the stacked multi-source path (push only until tuned)
    double stack_beta = 24.0;
    int64_t stack_handoff = 1 << 20;  // push levels of rpq_multi_source with this many edges (and V/16) run as phase kernels (0 = never)
    int32_t max_batch = 256;
    int64_t mem_budget = 0;  // 0 = a quarter of the free device memory at first use
    int32_t max_slots = 128;
    int64_t large_pairs = 1 << 21;  // served path: queries above this many reached pairs count as large
    int32_t large_slots = 0;        // concurrent served queries while recent queries are large (0: one at a time, single-query kernel)
    int32_t serve_stack_min = 32;   // waiting served requests of one NFA that run as one stacked group (0 = never)
    int64_t serve_group_wait_us = 200;  // served path: a burst of one NFA's requests waits this long for more before slots take it (0 = never)
    int32_t serve_lanes = 2;        // served path: single-query executors for large queries (0 = none)
    int64_t serve_promote_pairs = 0;  // served path: a slot query that reaches more pairs moves to a lane (0 = never)
    int64_t rare_end_max = 0;       // rare-end plan of rpq_single_source for at most this many candidate endpoints (0 = off)
    int32_t grid_override = 0;
    int32_t plain_grid = 0;  // persistent single-query launch workgroups (0 = one per CU)
    bool coop_launch = false;  // hipLaunchCooperativeKernel for the persistent single-query kernel
    std::recursive_mutex mu;
    // cached query constants of the single-query path
    rpq::QueryView qv{};
    std::vector<uint8_t> qbuf;
    uint64_t q_serial = 0;
    uint32_t q_force = ~0u, q_counters = ~0u;
    double q_alpha = -1, q_beta = -1;
    // Query constants of recent single-query calls stay in device memory
    // (qconst_dev is a bump arena of qconst_cap bytes, emptied when full), so
    // a query repeated with the same NFA handle and settings uploads nothing.
    struct QEntry {
        uint32_t force, counters;
        double alpha, beta;
        size_t off;
        int32_t nsym;
    };
    std::unordered_map<uint64_t, QEntry> qcache;  // by NFA serial
    size_t qarena_used = 0;
    // batched and served paths
    rpq::BatchState *batch = nullptr;
    // created by the first rpq_submit under serve_mu (not mu: a query the
    // scheduler runs holds mu, and submits must not wait for it)
    std::atomic<rpq::ServeState *> serve{nullptr};
    std::mutex serve_mu;
    // an executor made by exec_clone: the graph store belongs to this handle
    const rpq_graph *clone_of = nullptr;
};

namespace rpq {

rpq_status fail(rpq_status st, const char *fmt, ...);
// A persistent grid's share of its device's co-resident workgroups (see
// api.cpp): acquire() waits until `grid` workgroups of a kernel that fits
// blocks_per_cu times per compute unit can be resident next to every other
// persistent grid of this process; the destructor returns them.
class PersistentHold {
public:
    PersistentHold() = default;
    PersistentHold(const PersistentHold &) = delete;
    PersistentHold &operator=(const PersistentHold &) = delete;
    ~PersistentHold() { release(); }
    rpq_status acquire(int device, int grid, int blocks_per_cu);
    void release();

private:
    int device_ = -1;
    int64_t units_ = 0;
};
rpq_status hip_fail(hipError_t e, const char *what);
size_t build_qconst(const rpq_graph *g, const rpq_nfa *n, uint32_t force, uint32_t counters,
                    std::vector<uint8_t> &buf, int32_t *nsym_out);
size_t build_qconst_into(const rpq_graph *g, const rpq_nfa *n, uint32_t force, uint32_t counters, uint8_t *dst,
                         size_t cap, int32_t *nsym_out);
QueryView query_view(uint8_t *base, int32_t nsym);
rpq_status graph_upload(rpq_graph *g, const int64_t *label_ptr, const int32_t *src, const int32_t *dst);
// The single-query executor's state of a handle whose graph store is set.
rpq_status exec_alloc(rpq_graph *g);
// A second single-query executor on g's graph store (its own state arrays,
// staging, stream and query-constant cache, so that it can run a query while
// g or another executor runs one). It holds no part of the graph store: free
// it with exec_free before g. exec_sync_options copies the options of the
// plain path (pull thresholds, grid, launch kind) from g.
rpq_status exec_clone(const rpq_graph *g, rpq_graph **out);
void exec_sync_options(rpq_graph *c, const rpq_graph *g);
void exec_free(rpq_graph *c);
// Optional parts of a single-query call: a start set instead of one source
// (nsrc distinct vertices, already in g->pin_srcset) and the shortest-length
// output (V int32, device memory).
struct SingleExtra {
    int32_t nsrc = 0;
    int32_t *dist = nullptr;
};
rpq_status run_single(rpq_graph *g, const rpq_nfa *n, int32_t source, uint64_t *out, uint32_t flags,
                      rpq_stats *stats, const SingleExtra *ex = nullptr);
// Device memory for a stacked pass that the library does not allocate (see
// rpq_multi_source_noalloc): bytes at base, and the co-resident grid of the
// stacked kernel per [QM == 32][G].
struct StackArena {
    uint8_t *base;
    size_t bytes;
    int grid[2][17];
};
struct StackParams;
size_t stacked_arena_layout(const rpq_graph *g, int32_t Q, int G, int32_t B, uint8_t *base, StackParams *p,
                            uint8_t **qconst, int32_t **srcs, uint64_t **out);
// With probe >= 0 (at most MAX_BATCH sources, one batch): out_bitmaps is
// host memory that receives ceil(n_sources / 64) words, bit i set when source
// i reaches the vertex `probe` in a final state, instead of the bitmaps.
rpq_status stacked_run(rpq_graph *g, const rpq_nfa *n, const int32_t *sources, int32_t n_sources,
                       uint64_t *out_bitmaps, uint32_t flags, rpq_stats *stats, const char *who,
                       const StackArena *ar, int32_t probe = -1);
void serve_shutdown(rpq_graph *g);
bool serve_pending(rpq_graph *g);
// Slots the served path's engine admits queries into (0 before it exists).
int64_t serve_slots(rpq_graph *g);
// Lanes the served path has made (0 before its first large-query period).
int64_t serve_lane_count(rpq_graph *g);
void batch_free(rpq_graph *g);
// Clears the outputs of *st and keeps its caller-supplied input fields.
void stats_reset(rpq_stats *st);
// Fills the per-level outputs of *st (level_counts, level_us, level_frontier,
// level_edges) from `nrec` host copies of the device's per-level records
// (LVL_STRIDE words each; record `levels` carries only the end clock).
// Returns the sum of |M_n| over the copied levels.
int64_t stats_levels(rpq_stats *st, const uint64_t *lvl, uint32_t nrec, uint32_t levels);

}  // namespace rpq
