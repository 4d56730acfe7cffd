// Host-side construction of the graph store: the per-label Boolean
// decomposition {G^a} of Sec. 3 (Defs 3.7-3.8), kept for both directions
// (G^a and its transpose G^{a^-} = (G^a)^T) in a doubly-compressed form:
// per label only the vertices that have l-edges get a row, and a rank bitmap
// maps a vertex to its row in constant time. Duplicate entries are merged.
#include "graph_build.h"

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

namespace rpq {

template <typename F>
static void parallel_dynamic(int64_t n, F f) {
    unsigned nt = std::thread::hardware_concurrency();
    if (nt == 0) nt = 1;
    if (nt > 32) nt = 32;
    if (n < 2) nt = 1;
    std::atomic<int64_t> next{0};
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; t++)
        th.emplace_back([&] {
            for (int64_t i; (i = next.fetch_add(1)) < n;) f(i);
        });
    for (auto &x : th) x.join();
}

void build_direction(int32_t V, const int32_t *a, const int32_t *b, const int64_t *label_ptr, int32_t L,
                     uint32_t col_offset, HostDir &out) {
    const int64_t nw = (static_cast<int64_t>(V) + 63) / 64;
    std::vector<std::vector<uint64_t>> keys(static_cast<size_t>(L));
    out.label_edges.assign(static_cast<size_t>(L), 0);
    out.label_rows.assign(static_cast<size_t>(L), 0);
    // sort each label's (row, neighbour) pairs; biggest labels first
    std::vector<int32_t> order(static_cast<size_t>(L));
    for (int32_t l = 0; l < L; l++) order[l] = l;
    std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return label_ptr[x + 1] - label_ptr[x] > label_ptr[y + 1] - label_ptr[y];
    });
    parallel_dynamic(L, [&](int64_t i) {
        const int32_t l = order[i];
        std::vector<uint64_t> &k = keys[l];
        const int64_t lo = label_ptr[l], hi = label_ptr[l + 1];
        k.resize(static_cast<size_t>(hi - lo));
        for (int64_t e = lo; e < hi; e++)
            k[e - lo] = (static_cast<uint64_t>(static_cast<uint32_t>(a[e])) << 32) | static_cast<uint32_t>(b[e]);
        std::sort(k.begin(), k.end());
        k.erase(std::unique(k.begin(), k.end()), k.end());
        int64_t rows = 0;
        for (size_t j = 0; j < k.size(); j++)
            if (j == 0 || (k[j] >> 32) != (k[j - 1] >> 32)) rows++;
        out.label_edges[l] = static_cast<int64_t>(k.size());
        out.label_rows[l] = rows;
    });
    out.rbase.assign(static_cast<size_t>(L), 0);
    std::vector<int64_t> cbase(static_cast<size_t>(L) + 1, 0);
    uint64_t rtotal = 0;
    for (int32_t l = 0; l < L; l++) {
        out.rbase[l] = rtotal;
        rtotal += static_cast<uint64_t>(out.label_rows[l]) + 1;
        cbase[l + 1] = cbase[l] + out.label_edges[l];
    }
    out.E = cbase[L];
    out.rowptr.assign(rtotal, 0);
    out.rowvert.assign(rtotal, static_cast<uint32_t>(V));
    out.col.assign(static_cast<size_t>(out.E), 0);
    out.rankw.assign(static_cast<size_t>(L) * nw, RankWord{0, 0, 0});
    parallel_dynamic(L, [&](int64_t i) {
        const int32_t l = order[i];
        const std::vector<uint64_t> &k = keys[l];
        RankWord *rw = out.rankw.data() + static_cast<size_t>(l) * nw;
        uint32_t *rp = out.rowptr.data() + out.rbase[l];
        uint32_t *rv = out.rowvert.data() + out.rbase[l];
        uint32_t *c = out.col.data() + cbase[l];
        int64_t row = 0;
        for (size_t j = 0; j < k.size(); j++) {
            const uint32_t v = static_cast<uint32_t>(k[j] >> 32);
            if (j == 0 || (k[j] >> 32) != (k[j - 1] >> 32)) {
                rw[v >> 6].bits |= 1ull << (v & 63);
                rv[row] = v;
                rp[row++] = col_offset + static_cast<uint32_t>(cbase[l] + j);
            }
            c[j] = static_cast<uint32_t>(k[j]);
        }
        rp[row] = col_offset + static_cast<uint32_t>(cbase[l] + k.size());
        uint32_t r = 0;
        for (int64_t w = 0; w < nw; w++) {
            rw[w].rank = r;
            r += static_cast<uint32_t>(__builtin_popcountll(rw[w].bits));
        }
        std::vector<uint64_t>().swap(keys[l]);
    });
}

}  // namespace rpq
