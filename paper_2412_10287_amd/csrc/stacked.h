// Stacked multi-source traversal: B sources under one NFA in one traversal.
#pragma once

#include "rpq_internal.h"

namespace rpq {

// Every vertex v carries, per state q, a row of B source bits stored as G
// 64-bit words (G = ceil(B/64)): P, M[0], M[1] are [V][Q][G] uint64 arrays.
// sup[parity][v] is the set of states whose row in M[parity] is non-zero.
struct StackParams {
    GraphView g;
    QueryView qv;
    uint64_t *P;
    uint64_t *M[2];
    uint32_t *sup[2];
    int32_t *q[2];
    uint32_t *it_ebase, *it_beg, *it_v, *it_u;  // push items: (vertex, symbol) rows
    uint32_t *tile_first;
    LevelRec *rec;
    GridBarrier *bar;
    uint32_t *status;        // [0] levels, [3] invariant violations
    uint64_t *cnt;           // [0] items, [1] scanned edges, [2] word updates, [3] active vertices
    int64_t *lvl_pairs;      // |M_n| summed over sources, n < LVL_COUNT_CAP
    uint64_t *out;           // B bitmaps of nwords words
    const int32_t *sources;  // B vertex ids
    uint64_t item_cap, tile_cap;
    int64_t nwords;
    int32_t B, Q, V;
};

hipError_t launch_stacked(int G, const StackParams &p, int grid, hipStream_t s);
int stacked_grid(int G);

}  // namespace rpq
