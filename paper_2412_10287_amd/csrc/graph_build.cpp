// Host-side construction of the graph store: per direction, every vertex's
// incident edges grouped by label ("segments") and sorted by neighbour, with
// duplicates merged. This is the per-label Boolean decomposition {G^a} of
// Sec. 3 (Defs 3.7-3.8) kept in a vertex-major form, plus its transpose
// (G^{a^-} = (G^a)^T), so that one offset read per vertex reaches every label.
#include "graph_build.h"

#include <algorithm>
#include <thread>
#include <vector>

namespace rpq {

template <typename F>
static void parallel_for(int64_t n, F f) {
    unsigned nt = std::thread::hardware_concurrency();
    if (nt == 0) nt = 1;
    if (nt > 32) nt = 32;
    if (n < 100000) nt = 1;
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; t++) {
        int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
        th.emplace_back([=, &f] { f(lo, hi, t); });
    }
    for (auto &x : th) x.join();
}

// a[i] -> b[i] with label lab(i); keys grouped by a, sorted by (label, b).
void build_direction(int32_t V, int64_t E, const int32_t *a, const int32_t *b, const int64_t *label_ptr,
                     int32_t L, HostDir &out) {
    std::vector<int64_t> off(static_cast<size_t>(V) + 1, 0);
    for (int64_t i = 0; i < E; i++) off[a[i] + 1]++;
    for (int32_t v = 0; v < V; v++) off[v + 1] += off[v];
    std::vector<uint64_t> key(static_cast<size_t>(E));
    {
        std::vector<int64_t> fill(off.begin(), off.end() - 1);
        for (int32_t l = 0; l < L; l++)
            for (int64_t i = label_ptr[l]; i < label_ptr[l + 1]; i++)
                key[fill[a[i]]++] = (static_cast<uint64_t>(l) << 32) | static_cast<uint32_t>(b[i]);
    }
    // sort + dedupe each vertex's keys; count distinct edges and labels
    std::vector<int64_t> nedge(static_cast<size_t>(V)), nseg(static_cast<size_t>(V));
    parallel_for(V, [&](int64_t lo, int64_t hi, unsigned) {
        for (int64_t v = lo; v < hi; v++) {
            uint64_t *k0 = key.data() + off[v], *k1 = key.data() + off[v + 1];
            std::sort(k0, k1);
            uint64_t *ke = std::unique(k0, k1);
            nedge[v] = ke - k0;
            int64_t s = 0;
            for (uint64_t *k = k0; k < ke; k++)
                if (k == k0 || (k[0] >> 32) != (k[-1] >> 32)) s++;
            nseg[v] = s;
        }
    });
    out.vseg.assign(static_cast<size_t>(V) + 1, 0);
    std::vector<int64_t> eoff(static_cast<size_t>(V) + 1, 0);
    for (int32_t v = 0; v < V; v++) {
        out.vseg[v + 1] = out.vseg[v] + static_cast<uint32_t>(nseg[v]);
        eoff[v + 1] = eoff[v] + nedge[v];
    }
    const int64_t S = out.vseg[V];
    out.E = eoff[V];
    out.seg_lab.assign(static_cast<size_t>(S), 0);
    out.seg_beg.assign(static_cast<size_t>(S) + 1, 0);
    out.col.assign(static_cast<size_t>(out.E), 0);
    out.seg_beg[S] = static_cast<uint32_t>(out.E);
    parallel_for(V, [&](int64_t lo, int64_t hi, unsigned) {
        for (int64_t v = lo; v < hi; v++) {
            const uint64_t *k0 = key.data() + off[v];
            int64_t e = eoff[v];
            int64_t s = out.vseg[v];
            for (int64_t j = 0; j < nedge[v]; j++) {
                const uint64_t k = k0[j];
                if (j == 0 || (k >> 32) != (k0[j - 1] >> 32)) {
                    out.seg_lab[s] = static_cast<uint32_t>(k >> 32);
                    out.seg_beg[s] = static_cast<uint32_t>(e);
                    s++;
                }
                out.col[e++] = static_cast<uint32_t>(k);
            }
        }
    });
    out.label_edges.assign(static_cast<size_t>(L), 0);
    for (int64_t s = 0; s < S; s++) out.label_edges[out.seg_lab[s]] += out.seg_beg[s + 1] - out.seg_beg[s];
}

}  // namespace rpq
