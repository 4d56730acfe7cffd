// Internal structures shared by the host runtime and the HIP kernels of librpq.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpq {

constexpr int OUT = 0;  // adjacency G^a: row v holds the w with v -> w
constexpr int IN = 1;   // transpose (G^a)^T: row v holds the w with w -> v

constexpr int MAX_STATES = 32;
constexpr int MAX_SYMS = 256;              // distinct symbols one query may use
constexpr uint32_t REC_RING = 1024;        // level records kept in a ring
constexpr uint32_t LVL_COUNT_CAP = 65536;  // levels whose statistics are kept
// Per-level statistics, LVL_STRIDE uint64 per level n < LVL_COUNT_CAP:
//   [0] |M_n| (pairs first reached at level n), [1] frontier vertices,
//   [2] push reservation (items << 32 | edges), [3] device clock (100 MHz
//   wall clock) when level n started; entry [3] of the level after the last
//   one holds the clock when the traversal ended; [4] device clock when the
//   level's select phase ended (0 where no separate select phase exists).
constexpr uint32_t LVL_STRIDE = 5;
constexpr int BLOCK = 512;                 // threads per workgroup (8 waves)
constexpr int TILE = 4 * BLOCK;            // push edges per tile (one workgroup iteration)
constexpr int SYM_BATCH = 4;               // row lookups issued together per vertex
// Persistent launches use at most this many workgroups per CU (the occupancy
// API allows 3 for this kernel): every workgroup is resident at once, and
// fewer workgroups make each grid barrier cheaper.
constexpr int PERSISTENT_BLOCKS_PER_CU = 1;
constexpr int MAX_XCD = 16;

struct RankWordD {
    uint64_t bits;
    uint32_t rank;
    uint32_t pad;
};

// Device-resident graph store (label-major, both directions). For label l and
// direction d, vertex v has a row iff bit (v & 63) of rankw[(d*L + l)*nwords +
// (v >> 6)] is set; the row number is that word's rank plus the set bits below
// v, and its neighbours are col[rowptr[rbase[d][l] + row] .. rowptr[... + 1]).
struct GraphView {
    const RankWordD *rankw;
    const uint32_t *rowptr;
    const uint32_t *rowvert;  // vertex of each row (indexed like rowptr)
    const uint32_t *col;
    uint64_t ncol;   // entries of col (both directions)
    int64_t nwords;  // rank words per (direction, label)
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
    uint32_t force;      // 1 = push only, 2 = pull from level 0
    uint64_t e_rel;      // edges under the used symbols
    float alpha;         // push->pull threshold (0 = never pull)
    float beta;          // pull->push threshold
    uint32_t counters;   // 1 = accumulate the algorithmic counters
    uint32_t pad;
    uint32_t succ_any[MAX_STATES];  // OR over used symbols of succ[u][q]
};

// Layout of the device query-constant block: QHeader, then
//   symmask[32][4]                           (uint64: per state, the used
//                                             symbols with a transition out of it)
//   succ[nsym][32], pred[nsym][32]           (uint32 state sets)
//   push_w[nsym], pull_w[nsym]               (uint64 rank-word base)
//   push_r[nsym], pull_r[nsym]               (uint32 rowptr base)
//   pull_n[nsym]                             (uint32 rows in the pull direction)
// A forward symbol pushes along OUT rows and pulls along IN rows; an inverse
// symbol the other way round.
constexpr int SYM_WORDS = MAX_SYMS / 64;  // uint64 words of a symbol set

struct QueryView {
    const QHeader *h;
    const uint64_t *symmask;
    const uint32_t *succ;
    const uint32_t *pred;
    const uint64_t *push_w;
    const uint64_t *pull_w;
    const uint32_t *push_r;
    const uint32_t *pull_r;
    const uint32_t *pull_n;
};

struct QOffsets {
    size_t symmask, succ, pred, push_w, pull_w, push_r, pull_r, pull_n, end;
};

// Byte offsets of the tables in a query-constant block for nsym used symbols.
__host__ __device__ inline QOffsets qconst_offsets(size_t nsym) {
    QOffsets o;
    o.symmask = sizeof(QHeader);
    o.succ = o.symmask + MAX_STATES * SYM_WORDS * sizeof(uint64_t);
    o.pred = o.succ + nsym * MAX_STATES * sizeof(uint32_t);
    o.push_w = o.pred + nsym * MAX_STATES * sizeof(uint32_t);
    o.pull_w = o.push_w + nsym * sizeof(uint64_t);
    o.push_r = o.pull_w + nsym * sizeof(uint64_t);
    o.pull_r = o.push_r + nsym * sizeof(uint32_t);
    o.pull_n = o.pull_r + nsym * sizeof(uint32_t);
    o.end = o.pull_n + nsym * sizeof(uint32_t);
    return o;
}

// Bytes of the query-constant block for nsym used symbols.
__host__ __device__ inline size_t qconst_bytes(size_t nsym) { return qconst_offsets(nsym).end; }

// Query-constant blocks up to this size are copied into LDS by the
// persistent kernels (about 38 used symbols): the select phase's symbol
// tables are then one LDS access away instead of an L2 round trip.
constexpr size_t QC_LDS_BYTES = 12 * 1024;

// Table addresses of the block at `base` (host or device address).
__host__ __device__ inline QueryView qconst_view(const uint8_t *base, size_t nsym) {
    const QOffsets o = qconst_offsets(nsym);
    QueryView qv;
    qv.h = reinterpret_cast<const QHeader *>(base);
    qv.symmask = reinterpret_cast<const uint64_t *>(base + o.symmask);
    qv.succ = reinterpret_cast<const uint32_t *>(base + o.succ);
    qv.pred = reinterpret_cast<const uint32_t *>(base + o.pred);
    qv.push_w = reinterpret_cast<const uint64_t *>(base + o.push_w);
    qv.pull_w = reinterpret_cast<const uint64_t *>(base + o.pull_w);
    qv.push_r = reinterpret_cast<const uint32_t *>(base + o.push_r);
    qv.pull_r = reinterpret_cast<const uint32_t *>(base + o.pull_r);
    qv.pull_n = reinterpret_cast<const uint32_t *>(base + o.pull_n);
    return qv;
}

// One BFS level's bookkeeping (a ring of REC_RING entries). Every field that
// the whole grid updates with atomics sits on a 128-byte line of its own:
// atomics on one line are serialised (about 12 ns each on MI355X), so fields
// sharing a line would queue behind each other's updates.
struct alignas(128) LevelRec {
    uint32_t nq;          // frontier vertices (queue length) of this level
    uint32_t pad_nq[31];
    uint64_t sel;         // select phase: (items << 32) | push edges
    uint64_t pad_sel[15];
    uint64_t pairs;       // |M_n|
    uint64_t pad_pairs[15];
    uint32_t nfront;      // vertices with a non-empty frontier set
    uint32_t pad_nfront[31];
    uint32_t su;          // union of the frontier's state sets
    uint32_t pad_su[31];
    uint32_t mode;        // 0 push, 1 pull (decided when the level is expanded)
    uint32_t pad_mode;
    uint64_t hsel;        // (items << 32) | edges: stacked pull, the long rows deferred to the edge-balanced
                          // pass; single-query fused level, the workgroups' own items (statistics)
    uint64_t pad_hsel[14];
};

// Resets the fields of a level record (one thread).
__device__ __forceinline__ void rec_clear(LevelRec &r) {
    r.nq = 0;
    r.sel = 0;
    r.pairs = 0;
    r.nfront = 0;
    r.su = 0;
    r.mode = 0;
    r.hsel = 0;
}

// Two-level grid barrier state (see grid_barrier in kernels.hip).
struct GridBarrier {
    uint32_t reg[MAX_XCD];        // workgroups registered per XCD (this launch)
    uint32_t nreg;                // workgroups registered in total
    uint32_t gcount, ggen;        // XCD leaders arrived / generation
    uint32_t solo_n, solo_sel;    // where a run of small levels in workgroup 0 stopped
    uint32_t pad0[3];
    uint32_t status[7];           // the single-query launch's status words (StateView::status)
    uint32_t abort;               // a wait timed out; the launch ends early (after status: one copy reads both)
    uint32_t lcount[MAX_XCD][16]; // per-XCD arrivals (one 64-byte line each)
    uint32_t lgen[MAX_XCD][16];   // per-XCD generation
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
    uint64_t *lvl;        // per-level statistics (LVL_STRIDE words per level)
    uint64_t *out;        // output bitmap (device)
    uint32_t *status;     // [0] levels, [1] push levels, [2] pull levels, [3] invariant violations
    uint64_t *cnt;        // [0] product edges, [1] scans, [2] scanned edges, [3] active
    GridBarrier *bar;     // persistent-kernel barrier (zero at launch)
    GridBarrier *bar_next;  // the barrier of the next launch, zeroed by this one
    uint64_t item_cap;    // entries of the item arrays
    uint64_t tile_cap;    // entries of tile_first
    // Host-visible status (pinned host memory, or null): [0] levels, [1] push
    // levels, [2] pull levels, [3] 1 after an invariant violation, [4..5] |P|,
    // [6] 1 after a barrier abort, [7] hserial once the launch has finished.
    uint32_t *hstat;
    uint32_t hserial;
    // Levels in captured graphs (RPQ_GRAPH_LEVELS): [0] the level the next
    // select runs, [1] 1 once a level's expansion produced no candidates,
    // [2] the number of levels then.
    uint32_t *gctl;
};

struct Params {
    GraphView g;
    QueryView qv;
    StateView st;
    int32_t source;
    uint32_t nsrc;          // 0: one source (`source`); else the start set srcset[0..nsrc), distinct vertices
    const int32_t *srcset;  // device
    int32_t *dist;          // null, or V lengths of the shortest accepted walks (device; -1 = none)
};

// Launchers (kernels.hip). W is the state-word width in bytes: 1, 2 or 4.
hipError_t launch_persistent(int W, const Params &p, int grid, bool cooperative, hipStream_t s);
int persistent_grid(int W);          // co-resident workgroups for the persistent kernel
int occupancy_blocks_per_cu(int W);  // what the occupancy API reports
hipError_t launch_init(int W, const Params &p, hipStream_t s);
hipError_t launch_select(int W, const Params &p, uint32_t level, int grid, hipStream_t s);
hipError_t launch_expand(int W, const Params &p, uint32_t level, int grid, hipStream_t s);
hipError_t launch_final(int W, const Params &p, uint32_t nlevels, int grid, hipStream_t s);
// One captured level (select, expansion, advance) reading its Params from
// device memory and its level from p->st.gctl; every kernel of a level after
// the last returns at once.
hipError_t launch_level_g(int W, const Params *pdev, int grid, hipStream_t s);
hipError_t launch_fill(uint32_t *ptr, uint64_t words, uint32_t value, hipStream_t s);

}  // namespace rpq
