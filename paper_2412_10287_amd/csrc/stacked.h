// Stacked multi-source traversal: B sources under one NFA in one traversal.
#pragma once

#include "rpq_internal.h"

namespace rpq {

// Every vertex v carries, per state q, a row of B source bits stored as G
// 64-bit words (G = ceil(B/64)): P, M[0], M[1] are [V][Q][G] uint64 arrays.
//
// Level n works on the buffers of parity n & 1. While level n-1 expands, the
// rows M[n&1][w] collect candidate bits (not yet masked by P) and sup[n&1][w]
// the states that received any; the first writer of sup[n&1][w] appends w to
// q[n&1]. Level n's select then masks every candidate row by P, adds the new
// bits to P, and leaves in M[n&1][w] the frontier rows M_n and in sup[n&1][w]
// the frontier's state set (0 when every candidate bit was already visited).
// Work counters of one launch (p.cnt), filled when the query constants ask
// for counters; word updates are always counted.
enum {
    ST_CNT_SCANS = 0,   // (level, vertex, used symbol) with a non-empty successor set of the union state set
    ST_CNT_EDGES = 1,   // neighbours of those scans
    ST_CNT_UPDATES = 2, // (edge, transition, non-zero 64-bit source word) updates
    ST_CNT_ACTIVE = 3,  // (level, vertex) with a non-empty frontier column
    ST_CNT_WBYTES = 4,  // sum over active (level, v) of W(v) * (2 + neighbours scanned at v)
    ST_CNT_PE = 5,      // product edges summed over the sources
    ST_NCNT = 6
};

struct StackParams {
    GraphView g;
    QueryView qv;
    uint64_t *P;
    uint64_t *M[2];
    uint32_t *sup[2];
    int32_t *q[2];
    // work items: one (vertex, symbol) row each; it_s is the frontier state
    // set of the item's source vertex (push) or unused (pull)
    uint32_t *it_ebase, *it_beg, *it_v, *it_u, *it_s;
    uint32_t *tile_first;
    LevelRec *rec;
    GridBarrier *bar;
    uint32_t *status;        // [0] levels, [1] push levels, [2] pull levels, [3] invariant violations
    uint64_t *cnt;           // ST_NCNT work counters (ST_CNT_*), summed over the launch
    uint64_t *lvl;           // per-level statistics (LVL_STRIDE words), pairs summed over sources
    uint64_t *out;           // B bitmaps of nwords words; with a probe, G words: bit b = source b reaches the probe
    uint32_t probe;          // a vertex < V: only whether each source reaches it (in a final state) is written
    const int32_t *sources;  // B vertex ids
    uint64_t item_cap, tile_cap;
    int64_t nwords;
    int32_t B, Q, V;
    // Hand-off of large push levels to the phase kernels (k_st_expand,
    // k_st_compact, k_st_select): a launch of k_stacked stops before the
    // expansion of a push level with at least handoff_edges edges (0 = never)
    // and leaves its place in hand[]; a launch with hand[HAND_RESUME] set
    // continues at level hand[HAND_LEVEL], whose select is done.
    uint32_t *hand;
    uint64_t handoff_edges;
};

// Push levels with at least V / ST_SWEEP_DIV edges build the next queue in
// vertex order (st_compact) instead of appending while they expand.
constexpr uint32_t ST_SWEEP_DIV = 16;

// hand[] words (HAND_WORDS of them)
enum {
    HAND_EXIT = 0,    // out: 0 finished (final phase done), 1 stopped before a large push level
    HAND_LEVEL = 1,   // out: that level; in: the level to resume at
    HAND_RESUME = 2,  // in: 1 = resume (skip the start pairs, keep counters and statistics)
    HAND_NPUSH = 3,   // in/out: push levels so far
    HAND_NPULL = 4,   // in/out: pull levels so far
    HAND_LAST_LO = 5, // in: |M| of the last selected level (low, high words), for the level count
    HAND_LAST_HI = 6,
    HAND_WORDS = 16
};

// QM is the state bound the kernel is compiled for: 8 (every state set fits a
// byte; enables the pull direction) or 32.
hipError_t launch_stacked(int G, int QM, const StackParams &p, int grid, bool cooperative, hipStream_t s);
// Phase kernels for large push levels (no grid barrier: ordinary launches of
// as many workgroups as fit): the expansion of level n that marks the
// candidates' state sets (record: also write level n's statistics record),
// the vertex-ordered queue of level n + 1, and the select phase of level n.
hipError_t launch_st_expand(int G, int QM, const StackParams &p, uint32_t n, bool record, hipStream_t s);
hipError_t launch_st_compact(const StackParams &p, uint32_t n, hipStream_t s);
hipError_t launch_st_select(int G, int QM, const StackParams &p, uint32_t n, bool counters, hipStream_t s);
int stacked_grid(int G, int QM);
// Workgroups of the stacked kernel that fit on one compute unit (-1 on error).
int stacked_blocks_per_cu(int G, int QM);
// Device address of the fixed scratch array (RPQ_NOALLOC_SCRATCH_BYTES) on
// the current device.
hipError_t noalloc_scratch_address(void **ptr);

}  // namespace rpq
