/*
 * rpq.h - single-source two-way regular path queries on one MI355X (gfx950).
 *
 * The library evaluates the single-source reachability map of a two-way
 * regular path query (Sec. 2, Def. 2.6 and the SSR set): given an
 * edge-labelled graph (Def. 2.1), an epsilon-free NFA over labels and inverse
 * labels (Def. 2.4) and a source vertex, it returns every vertex u such that
 * some two-way walk from the source to u spells a word the NFA accepts.
 *
 * It does so by the level-synchronous traversal of Alg. 1 (Sec. 4): each level
 * computes M' = (sum over shared symbols a of (N^a)^T M G^a) masked by the
 * complement of P, then P = P + M', until M' is empty, and returns F P. Inverse
 * symbols use the transposed adjacency, G^{a^-} = (G^a)^T (Sec. 3). All work
 * after the graph is loaded runs in HIP kernels on the GPU.
 *
 * Conventions for every entry point:
 *  - Every call returns an rpq_status; no exception or abort crosses this
 *    interface. On failure rpq_last_error() describes the cause.
 *  - All input arrays are host memory unless a flag says otherwise; they are
 *    copied and the caller keeps ownership.
 *  - Vertex ids are 0-based int32 in [0, num_vertices). Bitmaps are
 *    rpq_bitmap_words(V) = ceil(V/64) uint64 words; vertex v is bit (v & 63) of
 *    word (v >> 6) (least significant bit first); pad bits are zero.
 *  - Handles are owned by the library until the matching *_free call.
 *  - Calls on one graph handle are serialized internally; different graph
 *    handles may be used from different threads. Persistent launches of the
 *    process on one GPU run side by side while their grids fit together (a
 *    per-device budget of co-resident workgroups) and wait otherwise.
 */
#ifndef RPQ_H
#define RPQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RPQ_OK = 0,
    RPQ_PENDING = 1,     /* rpq_poll: not finished yet */
    RPQ_EINVAL = -1,     /* invalid argument; nothing was done */
    RPQ_ENOMEM = -2,     /* host or device allocation failed */
    RPQ_EDEVICE = -3,    /* a HIP call failed; the handle may need to be freed */
    RPQ_EAGAIN = -4,     /* resource busy (e.g. graph freed with pending tickets) */
    RPQ_ENOTFOUND = -5,  /* unknown ticket or option */
    RPQ_ETIMEDOUT = -6   /* rpq_poll: timeout elapsed before completion */
} rpq_status;

typedef struct rpq_graph rpq_graph; /* device-resident graph store + query state */
typedef struct rpq_nfa rpq_nfa;     /* host-side NFA tables */
typedef uint64_t rpq_ticket;

/* Flags for the query entry points. */
#define RPQ_OUT_DEVICE 1u   /* out_bitmap(s) is device memory on the graph's GPU */
#define RPQ_COUNTERS 2u     /* fill the algorithmic work counters in rpq_stats */
#define RPQ_KERNEL_TIMING 4u /* time the expansion kernels with HIP events */
#define RPQ_FORCE_PUSH 8u   /* never use the pull direction (testing / tuning) */
#define RPQ_FORCE_PULL 16u  /* use the pull direction from level 1 on (testing / tuning) */
#define RPQ_HOST_LOOP 32u   /* drive levels from the host instead of one persistent launch */
#define RPQ_RARE_END 128u   /* rpq_single_source: the rare-end plan (see "rare_end_max"); RPQ_EINVAL
                                when it does not apply */
#define RPQ_GRAPH_LEVELS 64u /* single-query paths: levels as replays of a captured HIP graph of
                                16 levels (select, expansion, advance kernels), the end checked
                                once per replay; the graph is captured at first use per handle */

/*
 * Statistics of one query (or one batch). Input fields: level_counts may point
 * to a caller buffer of level_cap int64 that receives |M_n|, the number of
 * (state, vertex) pairs first reached at level n (the frontier sizes of
 * Alg. 1), for n < level_cap; it may be NULL.
 */
typedef struct {
    int64_t *level_counts;   /* in: optional buffer, level_cap entries */
    int32_t level_cap;       /* in */
    int32_t levels;          /* out: number of non-empty frontiers M_0..M_{levels-1} */
    int32_t push_levels;     /* out: levels expanded in the push direction */
    int32_t pull_levels;     /* out: levels expanded in the pull direction */
    int64_t visited_pairs;   /* out: |P|, reached (state, vertex) pairs */
    /* out, only with RPQ_COUNTERS (algorithmic work, independent of direction):
       product_edges = sum over reached (q,v) and symbols a of |succ_a(q)|*deg_a(v);
       scans = (level, vertex, used symbol) triples with a non-empty
       successor set, whether or not the vertex has neighbours under the
       symbol (a used symbol has a transition and a label some edge
       carries); scanned_edges = their neighbours;
       alg_bytes = sum over levels of (2w+8)*active + (8+(4+w)*deg) per scan,
       plus ceil(V/8), w the state-word bytes (1, 2, 4 for <= 8, 16, 32 states);
       active = (level, vertex) pairs with a non-empty frontier word. */
    int64_t product_edges, scans, scanned_edges, alg_bytes, active;
    double device_ms;        /* out: GPU time of the whole call (events); with
                                RPQ_KERNEL_TIMING on the persistent single-query
                                path, the kernel's time (= expand_ms) */
    double expand_ms;        /* out, with RPQ_KERNEL_TIMING: summed expansion-kernel time */
    int32_t expand_launches; /* out, with RPQ_KERNEL_TIMING */
    int32_t batch;           /* out: sources evaluated together */
    /* in: optional per-level outputs, each a caller buffer of level_cap
       entries (any may be NULL), filled for n < min(levels, level_cap) by
       rpq_single_source and rpq_multi_source (summed over a batch's sources,
       levels in lockstep; a call with several batches reports the last one):
       level_us: device time of level n in microseconds (GPU wall clock);
       level_frontier: vertices with a non-empty frontier state set at level n;
       level_edges: edges leaving the level-n frontier under symbols its state
       sets can take (the push work of level n, whichever direction ran);
       level_select_us: the part of level_us spent building the frontier and
       its work items, before the expansion (0 where not measured). */
    double *level_us;
    int64_t *level_frontier;
    int64_t *level_edges;
    double *level_select_us;
    /* out, rpq_multi_source: (edge, transition, non-zero 64-bit source word)
       updates the stacked expansion made (always filled; 0 elsewhere). With
       RPQ_COUNTERS the other work counters of a stacked call follow the
       batched model: scans are (level, vertex, used symbol) triples with a
       non-empty successor set of the union of the sources' frontier states
       at the vertex, active = (level, vertex) pairs with a non-empty frontier
       column, product_edges is summed over the sources, and alg_bytes =
       sum over active (level, v) of 8 + 2 W(v) plus 8 per scan plus
       (4 + W(v)) per scanned edge, plus B ceil(V/8), where W(v) is 4 bytes
       per non-zero 32-bit word of v's frontier column (source b in word
       b / 32 of each state's row). */
    int64_t updates;
    /* out, rpq_poll: host wall time from rpq_submit to the answer being
       ready, in milliseconds (0 elsewhere). A served query shares its
       launches with other queries, so it has no device time of its own and
       device_ms is 0 for it. */
    double latency_ms;
    /* out, rpq_single_source: 0 = the forward traversal from the source;
       1 = the rare-end plan (RPQ_RARE_END or option "rare_end_max"): one
       stacked traversal of the reversed automaton from the candidate
       endpoints; levels, push/pull levels, visited_pairs and times then
       describe that traversal and batch is the number of candidates. */
    int32_t plan;
} rpq_stats;

/* Number of uint64 words of a reachable-vertex bitmap over V vertices. */
int64_t rpq_bitmap_words(int32_t num_vertices);

/*
 * Build the device graph store from per-label COO edges (the Boolean
 * decomposition {G^a} of Sec. 3, Defs 3.7-3.8). Edges of label l are
 * (src[i] -> dst[i]) for i in [label_ptr[l], label_ptr[l+1]); label_ptr has
 * num_labels+1 entries with label_ptr[0] = 0. An edge with several labels
 * appears once per label. Duplicate entries are merged; self-loops are kept.
 * Both directions are stored (adjacency and transpose), as the two-way walks
 * need G^a and (G^a)^T.
 * Errors: RPQ_EINVAL for num_vertices < 1, num_labels < 1, a decreasing or
 * non-zero-based label_ptr, an id outside [0, num_vertices), more than
 * 2^31-1 distinct edges, or a NULL pointer with edges; RPQ_ENOMEM; RPQ_EDEVICE
 * when no usable GPU is present.
 */
rpq_status rpq_graph_load(int32_t num_vertices, int32_t num_labels, const int64_t *label_ptr,
                          const int32_t *src, const int32_t *dst, rpq_graph **out);
rpq_status rpq_graph_free(rpq_graph *g);
/* Graph facts: "num_vertices", "num_labels", "num_edges" (distinct), "device_bytes";
   "serve_slots": queries the served path holds at once, as its memory budget
   allowed when it started (0 before the first rpq_submit has been admitted);
   "serve_lanes": single-query executors the served path has made (0 before
   it needed one). */
rpq_status rpq_graph_info(const rpq_graph *g, const char *key, int64_t *value);

/*
 * Options on a graph handle (key, value):
 *  "stream"      hipStream_t (as an integer) the queries run on; 0 = the
 *                library's own stream. The stream must outlive its use.
 *  "pull_alpha"  push->pull switch: pull when the frontier's push edges exceed
 *                (edges of the query's symbols) / alpha; 0 disables pull.
 *  "pull_beta"   pull->push switch: back to push when the frontier has fewer
 *                than num_vertices / beta vertices.
 *  "persistent_grid"  workgroups of the persistent single-query launch
 *                (0 = one per CU; larger values are capped at that).
 *  "cooperative_launch"  1: start the persistent kernels (single-query and
 *                stacked multi-source) with
 *                hipLaunchCooperativeKernel, which guarantees that all its
 *                workgroups are resident at once; 0 (default): an ordinary
 *                launch, about 14 us faster per query on MI355X. The grid is
 *                sized to be resident on an otherwise idle GPU; if other work
 *                keeps some of its workgroups from starting for 5 s, the
 *                query fails with RPQ_EDEVICE (the grid barrier times out)
 *                instead of waiting further.
 *  "stacked_alpha", "stacked_beta"  the same two thresholds for
 *                rpq_multi_source (defaults 0, i.e. push only, and 24; pull
 *                needs <= 8 states).
 *  "max_batch"   largest number of sources stacked in one launch (<= 1024).
 *  "mem_budget"  device bytes the served path may use for query state.
 *  "max_slots"   concurrent queries in the served path.
 *  "rare_end_max"  rpq_single_source evaluates from the rare end when the
 *                query's candidate endpoints number at most this many (<=
 *                1024; default 0 = never): every vertex other than the source
 *                that a query can return is an endpoint of an edge whose
 *                symbol leads into a final state; when those vertices are
 *                few, one stacked traversal of the reversed automaton from
 *                all of them (Sec. 4's reversal; the evaluation-order hybrid
 *                of Secs 5.5 and 6) finds which of them reach the source. The
 *                answer is identical; the plan is not taken with per-level
 *                outputs, counters, or direction and level-driver flags.
 *  "serve_stack_min"  waiting served requests of one NFA handle that run as
 *                one stacked group (default 32; 0 = never).
 *  "serve_group_wait_us"  while at least serve_stack_min / 2 (and two)
 *                waiting requests share an NFA handle and the last request
 *                arrived less than this long ago, waiting requests are not
 *                admitted to slots, and a stacked group short of max_batch
 *                does not start unless its oldest request has waited 25
 *                times as long, so that a burst of one NFA's requests
 *                gathers into one group (default 200; 0 = at once; at most
 *                10^6).
 *  "large_query_pairs", "large_query_slots"  while the moving average of
 *                the reached (state, vertex) pairs of recently finished
 *                served queries exceeds large_query_pairs (default 2^21),
 *                at most large_query_slots run in slots at once (the state
 *                arrays of many large queries thrash the caches, and a few
 *                of them already fill the GPU); with large_query_slots 0
 *                (the default) such periods run requests through the
 *                single-query kernel once the slots have drained (the most
 *                efficient path per edge for large queries), on the lanes.
 *  "serve_lanes" single-query executors of the served path (default 2,
 *                at most 8; 0 = the scheduler thread runs such requests one
 *                at a time). Each has its own state arrays, stream and
 *                constant cache on the handle's graph store, and a thread.
 *  "serve_promote_pairs"  a query in a slot whose reached pairs pass this
 *                many moves to a lane and starts over there (default 0 =
 *                never; large-query periods apply instead).
 *  "stacked_handoff_edges"  rpq_multi_source runs push levels of at least
 *                this many edges (and V/16) as separate phase kernels with
 *                more waves per CU than the persistent kernel (default
 *                2^20; 0 = never). The answers are the same.
 * Errors: RPQ_ENOTFOUND for an unknown key, RPQ_EINVAL for a bad value.
 */
rpq_status rpq_set_option(rpq_graph *g, const char *key, int64_t value);
rpq_status rpq_get_option(const rpq_graph *g, const char *key, int64_t *value);

/*
 * Build an NFA (Sec. 2, Def. 2.4) from its per-symbol Boolean transition
 * matrices N^a in coordinate form (Sec. 4, Alg. 1 input). Symbol s <
 * num_labels is label s; s >= num_labels is the inverse of label
 * s - num_labels. Transitions of symbol s are (from[i] -> to[i]) for i in
 * [sym_ptr[s], sym_ptr[s+1]); sym_ptr has 2*num_labels+1 entries. start and
 * final_states list state ids (duplicates allowed). Symbols whose label the
 * graph lacks contribute nothing at query time (the shared-alphabet rule of
 * Alg. 1), which is not an error.
 * Errors: RPQ_EINVAL for num_states outside [1, 32], num_labels < 0, a state
 * id out of range, a decreasing sym_ptr, or NULL arrays with entries.
 */
rpq_status rpq_nfa_load(int32_t num_states, int32_t num_labels, const int64_t *sym_ptr,
                        const int32_t *from, const int32_t *to, const int32_t *start,
                        int32_t n_start, const int32_t *final_states, int32_t n_final,
                        rpq_nfa **out);
rpq_status rpq_nfa_free(rpq_nfa *n);

/*
 * One single-source query (Alg. 1 with the visited set initialised to the
 * start pairs, i.e. counting the zero-length walk). Blocking. out_bitmap
 * receives rpq_bitmap_words(V) words (host memory, or device memory with
 * RPQ_OUT_DEVICE). stats may be NULL.
 * Errors: RPQ_EINVAL for a NULL handle/output or a source outside
 * [0, num_vertices); RPQ_EDEVICE on a HIP failure.
 */
rpq_status rpq_single_source(rpq_graph *g, const rpq_nfa *n, int32_t source,
                             uint64_t *out_bitmap, uint32_t flags, rpq_stats *stats);

/*
 * Single-destination reachability (Sec. 2, the SDR map): every vertex s such
 * that some two-way walk from s to `target` spells a word the NFA accepts.
 * Evaluated as the single-source query of the reversed automaton (Sec. 4):
 * each transition turned around with its symbol inverted, start and final
 * sets swapped. Arguments, flags, output and errors as rpq_single_source.
 */
rpq_status rpq_single_destination(rpq_graph *g, const rpq_nfa *n, int32_t target, uint64_t *out_bitmap,
                                  uint32_t flags, rpq_stats *stats);

/*
 * Lengths of the shortest accepted walks from one source (the other semirings
 * Sec. 6 names as future work: min over walk lengths instead of the Boolean
 * OR). out_lengths receives num_vertices int32 (host memory, or device memory
 * with RPQ_OUT_DEVICE): entry v is the least length n of a two-way walk from
 * `source` to v whose word the NFA accepts, i.e. the least level n of Alg. 1
 * with v holding a final state in M_n (min over final states q_f of the
 * product-graph distance of (q_f, v); App. A: M_n holds exactly the pairs at
 * distance n), or -1 when no such walk exists. Entry v is >= 0 exactly when
 * rpq_single_source would set bit v. Other flags, stats and errors as
 * rpq_single_source.
 */
rpq_status rpq_single_source_lengths(rpq_graph *g, const rpq_nfa *n, int32_t source, int32_t *out_lengths,
                                     uint32_t flags, rpq_stats *stats);

/*
 * Reachability from a set of sources (Def. 2.6 allows a start set V_s): every
 * vertex u such that a two-way walk from some s in V_s to u spells a word the
 * NFA accepts, i.e. the union of the single-source answers. One traversal
 * starting from M_0 = Q_S x V_s; sources (host memory, n_sources entries)
 * may repeat. Level counts are those of that traversal (|M_n| = pairs at
 * distance n from the nearest start pair). Output, flags and errors as
 * rpq_single_source, plus RPQ_EINVAL for n_sources < 1.
 */
rpq_status rpq_source_set(rpq_graph *g, const rpq_nfa *n, const int32_t *sources, int32_t n_sources,
                          uint64_t *out_bitmap, uint32_t flags, rpq_stats *stats);

/*
 * Many sources under one NFA, stacked into one traversal (the multiple-source
 * direction of Sec. 6): every vertex carries one bit per (state, source). The
 * result of source i is identical to rpq_single_source's and is written to
 * out_bitmaps + i * rpq_bitmap_words(V). Sources may repeat. Blocking.
 * Errors: as rpq_single_source, plus RPQ_EINVAL for n_sources < 1.
 */
rpq_status rpq_multi_source(rpq_graph *g, const rpq_nfa *n, const int32_t *sources,
                            int32_t n_sources, uint64_t *out_bitmaps, uint32_t flags,
                            rpq_stats *stats);

/*
 * rpq_multi_source without allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). The same traversal, answers and statistics as
 * rpq_multi_source, but every piece of per-call device state (frontier,
 * visited and candidate rows, queues, work items, level records, barrier,
 * status words, query constants, the batch's sources, and the result bitmaps
 * when out_bitmaps is host memory) lives in one fixed array of
 * RPQ_NOALLOC_SCRATCH_BYTES bytes of device memory that the library owns:
 * each GPU holds its own copy from the first call on it until the process
 * ends. The call makes no hipMalloc, hipFree or other allocating call (the
 * graph store and its pinned staging buffer come from rpq_graph_load).
 * Every call on a GPU reuses that GPU's array and clears what must start at
 * zero; calls on one GPU are serialized inside the process (calls that
 * overlapped on one array would race). A batch needs
 * 3 * 8 * V * Q * G bytes of state rows (G = 64-source words per row, a power
 * of two >= ceil(B / 64), B = min(n_sources, max_batch)) plus about
 * 20 (V + rows) bytes of queues and work items, 2.7 MB of level records and
 * B * ceil(V / 64) * 8 bytes of results; a call whose first batch exceeds
 * the array fails with RPQ_EINVAL before any device work, and the message
 * gives both sizes. Other arguments, flags and errors as rpq_multi_source.
 */
#define RPQ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
rpq_status rpq_multi_source_noalloc(rpq_graph *g, const rpq_nfa *n, const int32_t *sources,
                                    int32_t n_sources, uint64_t *out_bitmaps, uint32_t flags,
                                    rpq_stats *stats);

/*
 * Served path. rpq_submit copies what it needs (the NFA may be freed after it
 * returns) and queues the query; a scheduler thread admits queued queries into
 * free slots while memory allows, advances all admitted queries level by level
 * in shared launches, and moves finished answers into a device-side result
 * pool (2 * slots entries). Thread-safe.
 * rpq_poll waits up to timeout_us microseconds (0 = just check, < 0 = forever):
 * RPQ_OK when finished (the bitmap copied to out_bitmap: host memory, or
 * device memory on the graph's GPU with RPQ_OUT_DEVICE; the ticket retired and
 * its pool entry freed), RPQ_PENDING if not finished and timeout_us == 0,
 * RPQ_ETIMEDOUT if the wait elapsed, RPQ_ENOTFOUND for an unknown ticket.
 * Finished answers hold their pool entry until polled; while every entry is
 * held, further answers are kept in host memory instead.
 * Requests of one NFA handle that wait together (at least "serve_stack_min"
 * of them, default 32) run as one stacked multi-source traversal, as
 * rpq_multi_source would (up to "max_batch" per group); their answers are the
 * same, and their statistics are the group's (levels, visited pairs) with
 * batch = the group size.
 */
rpq_status rpq_submit(rpq_graph *g, const rpq_nfa *n, int32_t source, rpq_ticket *out);
/*
 * rpq_submit with a deadline for the request to start: if it is still queued
 * deadline_us microseconds after this call (no slot, lane or group took it),
 * it is dropped and rpq_poll of its ticket returns RPQ_ETIMEDOUT with the
 * ticket retired (a later poll gives RPQ_ENOTFOUND). A request that has
 * started runs to completion. deadline_us <= 0: no deadline (rpq_submit).
 * Unlike a poll whose own wait elapsed (RPQ_ETIMEDOUT, ticket kept), the
 * message of rpq_last_error() then names the deadline.
 */
rpq_status rpq_submit_deadline(rpq_graph *g, const rpq_nfa *n, int32_t source, int64_t deadline_us,
                               rpq_ticket *out);
rpq_status rpq_poll(rpq_graph *g, rpq_ticket t, uint64_t *out_bitmap, uint32_t flags, rpq_stats *stats,
                    int64_t timeout_us);

/*
 * Autotuner (setting selection by measurement). Times every candidate setting
 * of one path on a sample of queries and keeps the fastest on the handle:
 *  RPQ_TUNE_PLAIN: queries nfas[i] from sources[i], i < n_queries, through
 *    rpq_single_source; tunes "persistent_grid" (workgroups of the persistent
 *    launch: one per CU, or a half, quarter or eighth of that) and the
 *    direction thresholds "pull_alpha" / "pull_beta".
 *  RPQ_TUNE_STACKED: nfas[0] from all n_queries sources through
 *    rpq_multi_source; tunes "stacked_alpha" / "stacked_beta", then, with
 *    the best of those, "stacked_handoff_edges" in {0 (no phase kernels),
 *    2^20, 2^22, 2^24} (levels below V/16 edges stay in the persistent
 *    kernel whatever the threshold).
 * Candidates: alpha in {0 (push only), 1, 2, 4, 8, 16, 64} x beta in
 * {4, 24, 128}. The time of a setting is the summed device time (HIP events)
 * of the sample after one warm-up pass with the handle's previous settings.
 * out receives the chosen values, their time and the previous settings'
 * time. Errors: RPQ_EINVAL for bad arguments, others as the query paths (the
 * previous settings are then kept).
 */
#define RPQ_TUNE_PLAIN 0
#define RPQ_TUNE_STACKED 1
typedef struct {
    int64_t grid;        /* persistent-launch workgroups chosen (0 = one per CU) */
    int64_t alpha, beta; /* direction thresholds chosen (alpha 0 = push only) */
    double best_ms;      /* device time of the sample with the chosen setting */
    double default_ms;   /* device time with the settings the handle had before */
    int32_t candidates;  /* settings timed */
    int64_t handoff_edges; /* stacked: "stacked_handoff_edges" chosen; plain: 0 */
} rpq_tuning;
rpq_status rpq_autotune(rpq_graph *g, int32_t path, const rpq_nfa *const *nfas, const int32_t *sources,
                        int32_t n_queries, rpq_tuning *out);

/* Thread-local description of the last failure on this thread. */
const char *rpq_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RPQ_H */
