// Multi-query engine: many queries (slots), each with its own NFA and source,
// advanced one level at a time in shared launches.
#pragma once

#include "rpq_internal.h"

namespace rpq {

constexpr size_t QC_STRIDE = 64 * 1024;  // bytes of query constants per slot (<= MAX_SYMS symbols)
constexpr int MW = 4;                     // state-word bytes of the multi-query engine

struct MultiParams {
    GraphView g;
    const uint8_t *qconst;   // slot s: qconst + s * QC_STRIDE (layout of build_qconst)
    uint32_t *P;             // slot s: P + s * swords (one 32-bit state word per vertex)
    uint32_t *M[2];          // frontier words by level parity, same layout
    uint32_t *q[2];          // combined frontier queues: (slot << vbits) | vertex
    // control block, copied to the host in one transfer per level:
    //   qlen[2] (queue lengths by parity), status (invariant violations),
    //   next_count[slots] (entries appended per slot this level),
    //   pairs[slots] (reached (state, vertex) pairs per slot, 8-byte aligned)
    uint32_t *ctl;
    uint32_t *qlen;
    uint32_t *status;
    uint32_t *next_count;
    uint64_t *pairs;
    uint64_t *sel;           // [2] select reservations by chunk parity: (items << 40) | edges
    uint64_t *it_ebase;      // items: first edge number
    uint32_t *it_beg;        // items: first col position
    uint32_t *it_mask;       // items: successor state set
    uint32_t *it_slot;       // items: slot
    uint32_t *tile_first;    // first item of each push tile
    uint64_t *out;           // extract: one bitmap per finished slot (nwords each)
    uint64_t swords;         // 32-bit words per slot array
    uint64_t item_cap, tile_cap, queue_cap;
    uint32_t slots;
    uint32_t vbits;          // bits of a vertex id in a queue entry
    int32_t V;
};

hipError_t multi_admit(const MultiParams &p, uint32_t parity, uint32_t n, const uint32_t *slot_src,
                       hipStream_t s);
hipError_t multi_select(const MultiParams &p, uint32_t parity, uint32_t lo, uint32_t hi, uint32_t clear_n,
                        int first_chunk, uint32_t chunk_id, int grid, hipStream_t s);
hipError_t multi_push(const MultiParams &p, uint32_t parity, uint32_t chunk_id, int grid, hipStream_t s);
// bytes of the control block for `slots` slots, and the offset of pairs[] in it
inline size_t multi_ctl_bytes(uint32_t slots) { return 16 + 4 * static_cast<size_t>(slots) + 8 + 8 * static_cast<size_t>(slots); }
inline size_t multi_pairs_offset(uint32_t slots) { return (16 + 4 * static_cast<size_t>(slots) + 7) & ~static_cast<size_t>(7); }
hipError_t multi_extract(const MultiParams &p, uint32_t nfin, const uint32_t *fin_slots, uint64_t nwords,
                         hipStream_t s);

}  // namespace rpq
