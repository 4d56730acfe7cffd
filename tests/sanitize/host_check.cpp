// Host code under the address, undefined-behaviour and thread sanitizers (a
// CPU build of its own; see test_sanitize.py): the graph-store builder of
// the library (build_direction, multithreaded) and the oracle (plain C) run
// on seeded random graphs, including empty labels, self-loops, duplicate
// entries and vertex counts around the 64-vertex rank-word boundary. Each
// result is checked against what its definition fixes (every input edge in
// exactly one row, rows sorted and free of duplicates, rank words counting
// the rows before them; the oracle's bitmap, distances and level counts
// agreeing with each other). Exit status 0 and "ok" when every check holds.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <set>
#include <tuple>
#include <vector>

#include "../../paper_2412_10287_amd/csrc/graph_build.h"

extern "C" {
typedef struct og_graph og_graph;
og_graph *og_new(int32_t nv, int32_t nl, const int64_t *label_ptr, const int32_t *src, const int32_t *dst);
void og_free(og_graph *g);
int32_t og_ssr(const og_graph *g, int32_t nq, int32_t nfa_nl, const int64_t *sym_ptr, const int32_t *tfrom,
               const int32_t *tto, const int32_t *start, int32_t nstart, const int32_t *fin, int32_t nfin,
               int32_t source, uint64_t *bitmap, int32_t *dist_out, int64_t *level_counts, int32_t level_cap,
               int64_t *counters, int32_t word_bytes);
}

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64() {  // xorshift64*
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * 0x2545f4914f6cdd1dull;
}
static int32_t below(int64_t n) { return static_cast<int32_t>(next_u64() % static_cast<uint64_t>(n)); }

static int failures = 0;
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            fprintf(stderr, "check failed: %s: ", #cond);  \
            fprintf(stderr, __VA_ARGS__);                  \
            fprintf(stderr, "\n");                         \
            failures++;                                    \
        }                                                  \
    } while (0)

// One direction: rows of label l are the vertices a with an l-edge, each
// row lists the distinct b in increasing order.
static void check_direction(int32_t V, int32_t L, const std::vector<int64_t> &lp, const std::vector<int32_t> &a,
                            const std::vector<int32_t> &b, uint32_t off, const rpq::HostDir &d) {
    const int64_t nwords = (V + 63) / 64;
    std::set<std::tuple<int32_t, int32_t, int32_t>> want;  // (label, a, b)
    for (int32_t l = 0; l < L; l++)
        for (int64_t i = lp[l]; i < lp[l + 1]; i++) want.insert({l, a[i], b[i]});
    CHECK(d.E == static_cast<int64_t>(want.size()), "E %lld distinct %zu", (long long)d.E, want.size());
    CHECK(d.rankw.size() == static_cast<size_t>(L * nwords), "rank words %zu", d.rankw.size());
    std::set<std::tuple<int32_t, int32_t, int32_t>> got;
    for (int32_t l = 0; l < L; l++) {
        uint32_t rank = 0;
        const uint64_t base = d.rbase[l];
        for (int64_t k = 0; k < nwords; k++) {
            const rpq::RankWord &rw = d.rankw[static_cast<size_t>(l * nwords + k)];
            CHECK(rw.rank == rank, "label %d word %lld rank %u want %u", l, (long long)k, rw.rank, rank);
            if (k == nwords - 1 && (V & 63))
                CHECK((rw.bits >> (V & 63)) == 0, "label %d: bits beyond V", l);
            for (int bit = 0; bit < 64; bit++) {
                if (!((rw.bits >> bit) & 1)) continue;
                const int32_t v = static_cast<int32_t>(k * 64 + bit);
                const uint64_t r = base + rank;
                CHECK(d.rowvert[r] == static_cast<uint32_t>(v), "label %d row %u vertex %u want %d", l, rank,
                      d.rowvert[r], v);
                const uint32_t s = d.rowptr[r], e = d.rowptr[r + 1];
                CHECK(s >= off && e > s, "label %d vertex %d: empty or misplaced row [%u, %u)", l, v, s, e);
                for (uint32_t p = s; p < e && p - off < d.col.size(); p++) {
                    const uint32_t w = d.col[p - off];
                    CHECK(w < static_cast<uint32_t>(V), "neighbour %u out of range", w);
                    if (p > s) CHECK(d.col[p - off - 1] < w, "row of %d (label %d) not strictly increasing", v, l);
                    got.insert({l, v, static_cast<int32_t>(w)});
                }
                rank++;
            }
        }
        CHECK(static_cast<int64_t>(rank) == d.label_rows[l], "label %d rows %u want %lld", l, rank,
              (long long)d.label_rows[l]);
    }
    CHECK(got == want, "edge sets differ (%zu against %zu)", got.size(), want.size());
}

int main() {
    const int32_t sizes[] = {1, 2, 63, 64, 65, 130, 1000};
    int graphs = 0, queries = 0;
    for (int32_t V : sizes) {
        for (int rep = 0; rep < 4; rep++) {
            const int32_t L = 1 + below(5);
            std::vector<int64_t> lp(L + 1, 0);
            std::vector<int32_t> src, dst;
            for (int32_t l = 0; l < L; l++) {
                const int64_t m = (l == 1) ? 0 : below(4 * static_cast<int64_t>(V) + 3);  // label 1 empty
                for (int64_t i = 0; i < m; i++) {
                    int32_t u = below(V), v = below(V);
                    if (i % 7 == 3) v = u;  // self-loop
                    src.push_back(u);
                    dst.push_back(v);
                    if (i % 5 == 1) {  // duplicate entry
                        src.push_back(u);
                        dst.push_back(v);
                    }
                }
                lp[l + 1] = static_cast<int64_t>(src.size());
            }
            rpq::HostDir out, in;
            rpq::build_direction(V, src.data(), dst.data(), lp.data(), L, 0, out);
            rpq::build_direction(V, dst.data(), src.data(), lp.data(), L, static_cast<uint32_t>(out.E), in);
            check_direction(V, L, lp, src, dst, 0, out);
            check_direction(V, L, lp, dst, src, static_cast<uint32_t>(out.E), in);
            graphs++;
            // the oracle on the same graph: a two-state automaton 0 -l-> 1,
            // 1 -l'-> 1 (l' possibly inverse), final state 1
            og_graph *og = og_new(V, L, lp.data(), src.data(), dst.data());
            CHECK(og != nullptr, "og_new failed");
            if (!og) continue;
            for (int q = 0; q < 3; q++) {
                const int32_t nsym = 2 * L;
                const int32_t s1 = below(nsym), s2 = below(nsym);
                std::vector<int64_t> sp(nsym + 1, 0);
                std::vector<int32_t> fr, to;
                for (int32_t s = 0; s < nsym; s++) {
                    if (s == s1) { fr.push_back(0); to.push_back(1); }
                    if (s == s2) { fr.push_back(1); to.push_back(1); }
                    sp[s + 1] = static_cast<int64_t>(fr.size());
                }
                const int32_t start = 0, fin = 1, source = below(V);
                std::vector<uint64_t> bm((V + 63) / 64, 0);
                std::vector<int32_t> dist(2 * static_cast<size_t>(V), 0);
                std::vector<int64_t> lc(4 * static_cast<size_t>(V) + 4, 0);
                int64_t cnt[5] = {0, 0, 0, 0, 0};
                const int32_t nl = og_ssr(og, 2, L, sp.data(), fr.data(), to.data(), &start, 1, &fin, 1, source,
                                          bm.data(), dist.data(), lc.data(), static_cast<int32_t>(lc.size()), cnt, 1);
                CHECK(nl >= 1, "og_ssr returned %d", nl);
                int64_t reached = 0, sum = 0;
                for (int32_t v = 0; v < V; v++) {
                    const bool bit = (bm[v >> 6] >> (v & 63)) & 1;
                    // state-major distances: the final state's entry decides the bit
                    const int32_t df = dist[static_cast<size_t>(fin) * V + v];
                    CHECK(bit == (df >= 0), "vertex %d: bit %d, final distance %d", v, bit, df);
                    for (int32_t st = 0; st < 2; st++) reached += dist[static_cast<size_t>(st) * V + v] >= 0;
                }
                for (int32_t k = 0; k < nl && k < static_cast<int32_t>(lc.size()); k++) sum += lc[k];
                CHECK(sum == reached, "level counts %lld, reached pairs %lld", (long long)sum, (long long)reached);
                CHECK(dist[static_cast<size_t>(start) * V + source] == 0, "source distance");
                queries++;
            }
            og_free(og);
        }
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("ok: %d graphs, %d oracle queries\n", graphs, queries);
    return 0;
}
