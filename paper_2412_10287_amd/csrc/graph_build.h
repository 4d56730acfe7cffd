#pragma once
#include <stdint.h>

#include <vector>

namespace rpq {

// One 64-vertex block of a label's row-presence bitmap plus the number of
// present rows before it (rank), so the row of vertex v is
// rank + popcount(bits below v).
struct RankWord {
    uint64_t bits;
    uint32_t rank;
    uint32_t pad;
};

// Label-major store of one direction: for every label l, the rows (vertices
// with at least one l-edge in this direction) as a rank bitmap, their
// neighbour ranges (rowptr) and the neighbours (col), duplicates removed.
struct HostDir {
    std::vector<RankWord> rankw;      // L * nwords
    std::vector<uint32_t> rowptr;     // per label: rows+1 entries, positions in col
    std::vector<uint32_t> rowvert;    // same indexing as rowptr: the vertex of each row (V after the last)
    std::vector<uint64_t> rbase;      // per label: first rowptr entry
    std::vector<uint32_t> col;        // neighbours, label-major
    std::vector<int64_t> label_edges; // distinct edges per label
    std::vector<int64_t> label_rows;  // rows per label
    int64_t E = 0;
};

// Edges a[i] -> b[i] of label l for i in [label_ptr[l], label_ptr[l+1]).
// col positions are offset by col_offset (so two directions can share one array).
void build_direction(int32_t V, const int32_t *a, const int32_t *b, const int64_t *label_ptr, int32_t L,
                     uint32_t col_offset, HostDir &out);

}  // namespace rpq
