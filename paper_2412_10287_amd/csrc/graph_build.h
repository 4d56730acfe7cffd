#pragma once
#include <stdint.h>

#include <vector>

namespace rpq {

struct HostDir {
    std::vector<uint32_t> vseg;     // V+1 segment offsets
    std::vector<uint32_t> seg_lab;  // label of each segment
    std::vector<uint32_t> seg_beg;  // first col position of each segment (+ sentinel)
    std::vector<uint32_t> col;      // neighbour ids
    std::vector<int64_t> label_edges;  // distinct edges per label
    int64_t E = 0;                  // distinct edges
};

void build_direction(int32_t V, int64_t E, const int32_t *a, const int32_t *b, const int64_t *label_ptr,
                     int32_t L, HostDir &out);

}  // namespace rpq
