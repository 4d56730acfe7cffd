// Internal structures shared by the host runtime and the HIP kernels of librpq.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpq {

constexpr int OUT = 0;  // adjacency G^a: edges v -> w stored at v
constexpr int IN = 1;   // transpose (G^a)^T: edges w -> v stored at v

constexpr int MAX_STATES = 32;
constexpr int MAX_SYMS = 256;          // distinct (label, direction) symbols one query may use
constexpr uint32_t REC_RING = 1024;    // level records kept in a ring
constexpr uint32_t LVL_COUNT_CAP = 65536;  // per-level pair counts kept for statistics
constexpr int BLOCK = 512;             // threads per workgroup (8 waves)
constexpr int TILE = 4 * BLOCK;        // push edges per tile (one workgroup iteration)
// Persistent launches use at most this many workgroups per CU: 16 of the 28
// wave slots a CU offers this kernel, so every workgroup is resident at once.
constexpr int PERSISTENT_BLOCKS_PER_CU = 2;

// Device-resident graph: per direction, a vertex-major "segment" layout.
// Vertex v owns segments [vseg[v], vseg[v+1]); segment s holds the neighbours
// of v under one label, seg_lab[s], at col[seg_beg[s] .. seg_beg[s+1]).
// Both directions share one col array (IN segments start after the E OUT ones).
struct GraphView {
    const uint32_t *vseg[2];
    const uint32_t *seg_lab[2];
    const uint32_t *seg_beg[2];
    const uint32_t *col;
    int32_t V;
    int32_t L;
};

// Query constants (device copy, written once per query from host memory).
// Symbol tables are indexed by the query's used-symbol number u.
struct QHeader {
    uint32_t Q;          // states
    uint32_t nsym;       // used symbols (label present in graph, has transitions)
    uint32_t smask;      // start states
    uint32_t fmask;      // final states
    uint32_t inmask;     // states with an incoming transition on a used symbol
    uint32_t pad0;
    uint64_t e_rel;      // edges under the used symbols (both directions as used)
    float alpha;         // push->pull threshold (0 = never pull)
    float beta;          // pull->push threshold
    uint32_t force;      // 1 = push only, 2 = pull from level 1
    uint32_t counters;   // 1 = accumulate the algorithmic counters
    uint32_t succ_any[MAX_STATES];  // OR over used symbols of succ[u][q]
};

// Layout of the device query-constant block: QHeader, then succ[nsym][32],
// pred[nsym][32] (uint32), then lab2sym[2][L] (int16; -1 = unused).
struct QueryView {
    const QHeader *h;
    const uint32_t *succ;
    const uint32_t *pred;
    const int16_t *l2s[2];  // push view: OUT segment label -> forward symbol,
                            // IN segment label -> inverse symbol
};

// One BFS level's bookkeeping (a ring of REC_RING entries).
struct LevelRec {
    uint32_t nq;          // frontier vertices (queue length) of this level
    uint32_t su;          // union of the frontier's state sets
    uint64_t pairs;       // |M_n|
    uint64_t sel;         // select phase: (items << 32) | push edges
    uint32_t mode;        // 0 push, 1 pull (decided when the level is expanded)
    uint32_t pad;
};

// Software grid barrier state (see grid_barrier in kernels.hip).
struct GridBarrier {
    uint32_t count;  // workgroups arrived at the current barrier
    uint32_t gen;    // barrier generation
    uint32_t abort;  // set when a wait timed out; the launch then ends early
    uint32_t pad;
};

// Per-query mutable device state.
struct StateView {
    uint32_t *P;          // visited, one state word per vertex (sub-word packed)
    uint32_t *M[2];       // frontier words: current / next by level parity
    int32_t *q[2];        // frontier vertex queues by level parity
    uint32_t *it_ebase;   // push items: first edge number
    uint32_t *it_beg;     // push items: first col position
    uint32_t *it_mask;    // push items: successor state set
    uint32_t *tile_first; // first item of each push tile
    LevelRec *rec;        // REC_RING records
    int64_t *lvl_pairs;   // |M_n| for n < LVL_COUNT_CAP
    uint64_t *out;        // output bitmap (device)
    uint32_t *status;     // [0] levels, [1] push levels, [2] pull levels
    uint64_t *cnt;        // [0] product edges, [1] scans, [2] scanned edges, [3] active
    GridBarrier *bar;     // persistent-kernel barrier (zero between launches)
};

struct Params {
    GraphView g;
    QueryView qv;
    StateView st;
    int32_t source;
};

// Launchers (kernels.hip). W is the state-word width in bytes: 1, 2 or 4.
hipError_t launch_persistent(int W, const Params &p, int grid, hipStream_t s);
int persistent_grid(int W);  // co-resident workgroups for the persistent kernel
int occupancy_blocks_per_cu(int W);  // what the occupancy API reports
hipError_t launch_init(int W, const Params &p, hipStream_t s);
hipError_t launch_select(int W, const Params &p, uint32_t level, int grid, hipStream_t s);
hipError_t launch_expand(int W, const Params &p, uint32_t level, int grid, hipStream_t s);
hipError_t launch_final(int W, const Params &p, uint32_t nlevels, int grid, hipStream_t s);
hipError_t launch_fill(uint32_t *ptr, uint64_t words, uint32_t value, hipStream_t s);

}  // namespace rpq
