// Multi-query engine: many queries (slots), each with its own NFA and source,
// advanced one level at a time in shared launches.
#pragma once

#include "rpq_internal.h"

namespace rpq {

constexpr size_t QC_STRIDE = 80 * 1024;  // bytes of query constants per slot (MAX_SYMS symbols fit)
constexpr int MW = 4;                     // state-word bytes of the multi-query engine
// select reservations pack items (high 26 bits) and edges (low 38 bits)
constexpr int SEL_SHIFT = 38;
constexpr uint64_t MAX_MULTI_ITEMS = 1ull << (64 - SEL_SHIFT);
constexpr uint32_t MAX_SLOTS_DEV = 256;   // slots the kernels' per-slot LDS tables hold

struct MultiParams {
    GraphView g;
    const uint8_t *qconst;   // slot s: qconst + s * QC_STRIDE (layout of build_qconst)
    uint32_t *P;             // slot s: P + s * swords (one 32-bit state word per vertex)
    uint32_t *M[2];          // frontier words by level parity, same layout
    uint32_t *q[2];          // combined frontier queues: (slot << vbits) | vertex
    // control block, copied to the host in one transfer per level:
    //   qlen[2] (queue lengths by parity), status (invariant violations),
    //   next_count[slots] (non-zero when the slot's next frontier is not empty),
    //   pairs[slots * PAIRS_STRIDE] (reached (state, vertex) pairs of slot s at
    //   s * PAIRS_STRIDE, one line per slot)
    uint32_t *ctl;
    uint32_t *qlen[2];        // next-queue lengths by parity (separate lines)
    uint32_t *status;
    uint32_t *next_count;
    uint64_t *pairs;
    uint64_t *sel;           // [2] select reservations by chunk parity: (items << SEL_SHIFT) | edges
    uint64_t *it_ebase;      // items: first edge number
    uint32_t *it_beg;        // items: first col position
    uint32_t *it_mask;       // items: successor state set
    uint32_t *it_slot;       // items: slot
    uint32_t *tile_first;    // first item of each push tile
    uint64_t *out;           // result pool: 3 * slots bitmaps of nwords words (the last slots stage spills)
    uint32_t *dead;          // per slot: non-zero = the query moved to a lane; its entries yield nothing
                             // (the select drops its candidate words) until the slot is admitted again
    uint64_t swords;         // 32-bit words per slot array
    uint64_t item_cap, tile_cap, queue_cap;
    uint32_t slots;
    uint32_t vbits;          // bits of a vertex id in a queue entry
    int32_t V;
};

// Admission of n requests from one staging upload: `stage` starts with n
// records (slot, source, byte offset of the request's query constants in
// stage, their size); the admit kernel copies each block into its slot's
// constants and sets the slot's start pairs.
constexpr size_t ADMIT_TABLE_BYTES = 16 * static_cast<size_t>(MAX_SLOTS_DEV);
hipError_t multi_admit(const MultiParams &p, uint32_t parity, uint32_t n, const uint8_t *stage, hipStream_t s);
hipError_t multi_select(const MultiParams &p, uint32_t parity, uint32_t lo, uint32_t hi, uint32_t clear_n,
                        int first_chunk, uint32_t chunk_id, int grid, hipStream_t s);
hipError_t multi_push(const MultiParams &p, uint32_t parity, uint32_t chunk_id, int grid, hipStream_t s);
// bytes of the control block for `slots` slots, and the offset of pairs[] in it
// Control block layout (bytes). Each field that kernels update heavily sits
// on a cache line of its own: the next queue's length (one atomic per
// workgroup and step of every push), the per-slot frontier flags (stored by
// appending lanes) and the per-slot pair counters (atomics at select time).
constexpr size_t CTL_LINE = 128;
constexpr size_t CTL_QLEN = 0;              // uint32 qlen[2], one line each
constexpr size_t CTL_STATUS = 2 * CTL_LINE; // uint32 invariant violations
constexpr size_t CTL_NEXT = 3 * CTL_LINE;   // uint32 next_count[slots]
inline size_t multi_pairs_offset(uint32_t slots) {
    return CTL_NEXT + ((4 * static_cast<size_t>(slots) + CTL_LINE - 1) / CTL_LINE) * CTL_LINE;
}
// pairs[] keeps each slot's counter on a line of its own (every workgroup of
// a select launch adds to the counters of the slots it saw)
constexpr size_t PAIRS_STRIDE = CTL_LINE / 8;  // uint64 entries per slot
inline size_t multi_ctl_bytes(uint32_t slots) {
    return multi_pairs_offset(slots) + CTL_LINE * static_cast<size_t>(slots);
}
// (slot, result-pool entry) pairs of the finished queries, passed by value
struct FinList {
    uint32_t n;
    uint32_t e[2 * MAX_SLOTS_DEV];
};
hipError_t multi_extract(const MultiParams &p, const FinList &fin, uint64_t nwords, hipStream_t s);
// Copies nwords 64-bit words from src to dst (device memory) and then stores
// seq into *flag (pinned host memory, as the device addresses it) once the
// copy is visible to every agent, so that a host can wait by polling the
// flag. done (device memory, zero between launches) counts finished
// workgroups.
hipError_t copy_signal(const uint64_t *src, uint64_t *dst, uint64_t nwords, uint32_t *done, uint32_t *flag,
                       uint32_t seq, hipStream_t s);
// Copies the control block (`words` 32-bit words) into host memory that the
// device addresses as `host` (pinned), on the stream of the level's kernels.
hipError_t multi_publish(const MultiParams &p, uint32_t *host, uint32_t words, hipStream_t s);

}  // namespace rpq
