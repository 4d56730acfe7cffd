/*
 * Reference oracle for single-source two-way regular path queries.
 *
 * TEST INFRASTRUCTURE ONLY. It is called by the test suite, by the smoke check
 * and by the benchmark's CPU-baseline leg, and by nothing on the product path.
 * It shares no code, header or table with the GPU library.
 *
 * What it computes is the plain definition of single-source reachability
 * (Sec. 2, Def. 2.6 and the SSR map): the set of vertices u such that some
 * two-way walk from the source to u spells a word accepted by the query's NFA
 * (walks may repeat vertices, Def. 2.2; the zero-length walk exists at every
 * vertex; a walk may use each edge forwards with its labels or backwards with
 * the inverted labels, Def. 2.3). By the correctness theorem of Sec. 4 (proved
 * in App. A) this is the set Alg. 1 returns, so the oracle does not follow
 * Alg. 1's matrix form: it is a first-in-first-out breadth-first search over
 * explicit (state, vertex) pairs of the product of the NFA and the graph
 * (Def. 2.5), with the inverse-label rule G^{a^-} = (G^a)^T of Sec. 3.
 *
 * FIFO order gives exact distances, so the pairs at distance n are exactly
 * the n-th frontier M_n of Alg. 1 (the invariant of App. A); the per-level
 * counts and the work counters below are derived from those distances.
 *
 * Readings taken where the paper is silent or inconsistent:
 *  - the visited set starts as the start pairs (the zero-length walk), as in
 *    Alg. 2's initialisation, not as the empty matrix of Alg. 1;
 *  - duplicate (edge, label) entries are merged (Boolean semantics);
 *  - NFA symbols whose label the graph does not have contribute nothing
 *    (the intersection of alphabets in Alg. 1's update);
 *  - at most 64 NFA states (the work counters use 64-bit state sets).
 *
 * Besides the answer it returns dist (the product-graph distance of every
 * (state, vertex) pair), from which the shortest accepted walk to v is the
 * least dist over the final states at v.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nv, nl;
    /* per vertex: outgoing (label, target) and incoming (label, origin)
       pairs, sorted by (label, neighbour), duplicates removed */
    int64_t *out_off, *in_off;
    int32_t *out_lab, *out_nbr, *in_lab, *in_nbr;
    /* has_edges[l] = 1 if at least one edge carries label l */
    uint8_t *has_edges;
} og_graph;

/* stable counting sort of idx[0..m) by key[idx[i]] in [0, nkeys) */
static int csort(int64_t m, int64_t *idx, const int32_t *key, int64_t nkeys) {
    int64_t *cnt = (int64_t *)calloc((size_t)nkeys + 1, sizeof(int64_t));
    int64_t *tmp = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!cnt || !tmp) { free(cnt); free(tmp); return -1; }
    for (int64_t i = 0; i < m; i++) cnt[key[idx[i]] + 1]++;
    for (int64_t k = 0; k < nkeys; k++) cnt[k + 1] += cnt[k];
    for (int64_t i = 0; i < m; i++) tmp[cnt[key[idx[i]]]++] = idx[i];
    memcpy(idx, tmp, (size_t)m * sizeof(int64_t));
    free(cnt); free(tmp);
    return 0;
}

/* Build one direction: group by `a`, then (label, b). Returns 0 on success. */
static int build_dir(int32_t nv, int32_t nl, int64_t m, const int32_t *a, const int32_t *b,
                     const int32_t *lab, int64_t **off_o, int32_t **lab_o, int32_t **nbr_o) {
    int64_t *idx = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!idx) return -1;
    for (int64_t i = 0; i < m; i++) idx[i] = i;
    /* least significant key first: neighbour, then label, then vertex */
    if (csort(m, idx, b, nv) || csort(m, idx, lab, nl) || csort(m, idx, a, nv)) { free(idx); return -1; }
    int64_t *off = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    int32_t *ol = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t *on = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!off || !ol || !on) { free(idx); free(off); free(ol); free(on); return -1; }
    int64_t k = 0;
    for (int64_t i = 0; i < m; i++) {
        int64_t e = idx[i];
        if (k > 0 && i > 0) {
            int64_t p = idx[i - 1];
            if (a[p] == a[e] && lab[p] == lab[e] && b[p] == b[e]) continue; /* duplicate */
        }
        ol[k] = lab[e];
        on[k] = b[e];
        off[a[e] + 1]++;
        k++;
    }
    for (int32_t v = 0; v < nv; v++) off[v + 1] += off[v];
    free(idx);
    *off_o = off; *lab_o = ol; *nbr_o = on;
    return 0;
}

void og_free(og_graph *g) {
    if (!g) return;
    free(g->out_off); free(g->in_off);
    free(g->out_lab); free(g->out_nbr); free(g->in_lab); free(g->in_nbr);
    free(g->has_edges);
    free(g);
}

/* Graph from per-label COO: edges of label l are [label_ptr[l], label_ptr[l+1]). */
og_graph *og_new(int32_t nv, int32_t nl, const int64_t *label_ptr, const int32_t *src,
                 const int32_t *dst) {
    if (nv < 1 || nl < 0 || !label_ptr) return NULL;
    int64_t m = label_ptr[nl];
    if (label_ptr[0] != 0 || m < 0) return NULL;
    int32_t *lab = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!lab) return NULL;
    for (int32_t l = 0; l < nl; l++) {
        if (label_ptr[l + 1] < label_ptr[l]) { free(lab); return NULL; }
        for (int64_t i = label_ptr[l]; i < label_ptr[l + 1]; i++) lab[i] = l;
    }
    for (int64_t i = 0; i < m; i++)
        if (src[i] < 0 || src[i] >= nv || dst[i] < 0 || dst[i] >= nv) { free(lab); return NULL; }
    og_graph *g = (og_graph *)calloc(1, sizeof(og_graph));
    if (!g) { free(lab); return NULL; }
    g->nv = nv; g->nl = nl;
    g->has_edges = (uint8_t *)calloc((size_t)(nl > 0 ? nl : 1), 1);
    if (!g->has_edges) { free(lab); og_free(g); return NULL; }
    for (int32_t l = 0; l < nl; l++) g->has_edges[l] = label_ptr[l + 1] > label_ptr[l];
    if (build_dir(nv, nl, m, src, dst, lab, &g->out_off, &g->out_lab, &g->out_nbr) ||
        build_dir(nv, nl, m, dst, src, lab, &g->in_off, &g->in_lab, &g->in_nbr)) {
        free(lab); og_free(g); return NULL;
    }
    free(lab);
    return g;
}

/* Neighbours of v under label l: forward (inv = 0) follows edges v -> w with
   label l; inverse (inv = 1) follows them backwards, i.e. edges w -> v. */
static void nbr_range(const og_graph *g, int32_t v, int32_t l, int inv, int64_t *lo, int64_t *hi) {
    const int64_t *off = inv ? g->in_off : g->out_off;
    const int32_t *lb = inv ? g->in_lab : g->out_lab;
    int64_t a = off[v], b = off[v + 1];
    /* first position with label >= l */
    int64_t x = a, y = b;
    while (x < y) { int64_t mid = x + (y - x) / 2; if (lb[mid] < l) x = mid + 1; else y = mid; }
    int64_t s = x;
    y = b;
    while (x < y) { int64_t mid = x + (y - x) / 2; if (lb[mid] <= l) x = mid + 1; else y = mid; }
    *lo = s; *hi = x;
}

int64_t og_num_edges(const og_graph *g, int inv) {
    return inv ? g->in_off[g->nv] : g->out_off[g->nv];
}

/*
 * One query from the start set V_s = sources[0..nsources) (Def. 2.6; a
 * single-source query has V_s = {source}): the search starts from every pair
 * of Q_S x V_s at distance 0, so dist is the distance from the nearest start
 * pair and the answer is the union of the sources' single-source answers.
 *   NFA: nq states; symbols s < nfa_nl are labels, s >= nfa_nl inverse labels
 *        of s - nfa_nl; transitions of symbol s are
 *        (tfrom[i] -> tto[i]), i in [sym_ptr[s], sym_ptr[s+1]).
 *   bitmap: ceil(V/64) words, bit v of word v>>6 (LSB first) = v reachable.
 *   dist (nullable): nq*V int32, dist[q*V + v] = BFS level of (q, v) or -1.
 *   level_counts (nullable): level_counts[n] = |M_n| for n < level_cap.
 *   counters (nullable, 5 int64): product edges out of the reached pairs,
 *        scans, graph edges scanned, algorithmic bytes for state words of
 *        word_bytes bytes, active (level, vertex) pairs. A scan is a
 *        (level n, vertex v, used symbol a) with succ_a(S_n(v)) non-empty,
 *        S_n(v) the states first reached at v at level n, whether or not v
 *        has a-neighbours: the byte model charges every scan the 8 bytes of
 *        the row-pointer pair that finds its neighbour range, plus 4 + w
 *        bytes per neighbour, plus 2w + 8 bytes per active (n, v).
 * Returns the number of levels (max distance + 1), or -1 on invalid input
 * or allocation failure.
 */
int32_t og_ssr_from(const og_graph *g, int32_t nq, int32_t nfa_nl, const int64_t *sym_ptr,
                    const int32_t *tfrom, const int32_t *tto, const int32_t *start, int32_t nstart,
                    const int32_t *fin, int32_t nfin, const int32_t *sources, int32_t nsources,
                    uint64_t *bitmap, int32_t *dist_out, int64_t *level_counts, int32_t level_cap,
                    int64_t *counters, int32_t word_bytes) {
    if (!g || nq < 1 || nq > 64 || nfa_nl < 0 || !sym_ptr || !sources || nsources < 1) return -1;
    for (int32_t i = 0; i < nsources; i++)
        if (sources[i] < 0 || sources[i] >= g->nv) return -1;
    const int32_t nv = g->nv;
    const int32_t nsym = 2 * nfa_nl;
    const int64_t nt = sym_ptr[nsym];
    for (int32_t i = 0; i < nstart; i++) if (start[i] < 0 || start[i] >= nq) return -1;
    for (int32_t i = 0; i < nfin; i++) if (fin[i] < 0 || fin[i] >= nq) return -1;
    for (int64_t i = 0; i < nt; i++)
        if (tfrom[i] < 0 || tfrom[i] >= nq || tto[i] < 0 || tto[i] >= nq) return -1;

    /* transitions grouped by origin state: (symbol, target) */
    int64_t *toff = (int64_t *)calloc((size_t)nq + 1, sizeof(int64_t));
    int32_t *tsym = (int32_t *)malloc((size_t)(nt > 0 ? nt : 1) * sizeof(int32_t));
    int32_t *ttgt = (int32_t *)malloc((size_t)(nt > 0 ? nt : 1) * sizeof(int32_t));
    int64_t cells = (int64_t)nq * nv;
    int32_t *dist = dist_out ? dist_out : (int32_t *)malloc((size_t)cells * sizeof(int32_t));
    int64_t *fifo = (int64_t *)malloc((size_t)cells * sizeof(int64_t));
    if (!toff || !tsym || !ttgt || !dist || !fifo) {
        free(toff); free(tsym); free(ttgt); free(fifo); if (!dist_out) free(dist); return -1;
    }
    for (int32_t s = 0; s < nsym; s++)
        for (int64_t i = sym_ptr[s]; i < sym_ptr[s + 1]; i++) toff[tfrom[i] + 1]++;
    for (int32_t q = 0; q < nq; q++) toff[q + 1] += toff[q];
    {
        int64_t *fill = (int64_t *)malloc((size_t)nq * sizeof(int64_t));
        if (!fill) { free(toff); free(tsym); free(ttgt); free(fifo); if (!dist_out) free(dist); return -1; }
        for (int32_t q = 0; q < nq; q++) fill[q] = toff[q];
        for (int32_t s = 0; s < nsym; s++)
            for (int64_t i = sym_ptr[s]; i < sym_ptr[s + 1]; i++) {
                tsym[fill[tfrom[i]]] = s;
                ttgt[fill[tfrom[i]]++] = tto[i];
            }
        free(fill);
    }

    for (int64_t i = 0; i < cells; i++) dist[i] = -1;
    int64_t head = 0, tail = 0;
    /* the start pairs Q_S x V_s at distance 0 (V_s = {source} for a
       single-source query; a repeated pair is queued once) */
    for (int32_t k = 0; k < nsources; k++)
        for (int32_t i = 0; i < nstart; i++) {
            int64_t c = (int64_t)start[i] * nv + sources[k];
            if (dist[c] < 0) { dist[c] = 0; fifo[tail++] = c; }
        }
    int32_t maxd = tail > 0 ? 0 : -1;
    while (head < tail) {
        int64_t c = fifo[head++];
        int32_t q = (int32_t)(c / nv), v = (int32_t)(c % nv);
        int32_t d = dist[c];
        for (int64_t t = toff[q]; t < toff[q + 1]; t++) {
            int32_t s = tsym[t];
            int inv = s >= nfa_nl;
            int32_t l = inv ? s - nfa_nl : s;
            if (l >= g->nl) continue; /* label absent from the graph */
            const int32_t *nb = inv ? g->in_nbr : g->out_nbr;
            int64_t lo, hi;
            nbr_range(g, v, l, inv, &lo, &hi);
            int32_t q2 = ttgt[t];
            for (int64_t k = lo; k < hi; k++) {
                int64_t c2 = (int64_t)q2 * nv + nb[k];
                if (dist[c2] < 0) {
                    dist[c2] = d + 1;
                    if (d + 1 > maxd) maxd = d + 1;
                    fifo[tail++] = c2;
                }
            }
        }
    }
    free(fifo);

    if (bitmap) {
        int64_t nw = ((int64_t)nv + 63) / 64;
        memset(bitmap, 0, (size_t)nw * sizeof(uint64_t));
        for (int32_t i = 0; i < nfin; i++)
            for (int32_t v = 0; v < nv; v++)
                if (dist[(int64_t)fin[i] * nv + v] >= 0) bitmap[v >> 6] |= 1ull << (v & 63);
    }
    int32_t nlev = maxd + 1;
    if (level_counts) {
        for (int32_t n = 0; n < level_cap; n++) level_counts[n] = 0;
        for (int64_t i = 0; i < cells; i++)
            if (dist[i] >= 0 && dist[i] < level_cap) level_counts[dist[i]]++;
    }
    if (counters) {
        /* successor sets per (symbol, state) for the symbols the NFA uses and
           some edge of the graph carries */
        int32_t *used = (int32_t *)malloc((size_t)(nsym > 0 ? nsym : 1) * sizeof(int32_t));
        int32_t nused = 0;
        for (int32_t s = 0; s < nsym; s++) {
            int32_t l = s >= nfa_nl ? s - nfa_nl : s;
            if (sym_ptr[s + 1] > sym_ptr[s] && l < g->nl && g->has_edges[l]) used[nused++] = s;
        }
        uint64_t *succ = (uint64_t *)calloc((size_t)(nused > 0 ? nused : 1) * nq, sizeof(uint64_t));
        for (int32_t u = 0; u < nused; u++)
            for (int64_t i = sym_ptr[used[u]]; i < sym_ptr[used[u] + 1]; i++)
                succ[(int64_t)u * nq + tfrom[i]] |= 1ull << tto[i];
        int64_t prod_edges = 0, scans = 0, scanned = 0, bytes = 0, active = 0;
        int32_t lv[64];
        uint64_t lm[64];
        for (int32_t v = 0; v < nv; v++) {
            int32_t nd = 0;
            for (int32_t q = 0; q < nq; q++) {
                int32_t d = dist[(int64_t)q * nv + v];
                if (d < 0) continue;
                int32_t j = 0;
                while (j < nd && lv[j] != d) j++;
                if (j == nd) { lv[nd] = d; lm[nd] = 0; nd++; }
                lm[j] |= 1ull << q;
            }
            if (nd == 0) continue;
            active += nd;
            bytes += (int64_t)nd * (2 * word_bytes + 8);
            for (int32_t u = 0; u < nused; u++) {
                int32_t s = used[u];
                int inv = s >= nfa_nl;
                int64_t lo, hi;
                nbr_range(g, v, inv ? s - nfa_nl : s, inv, &lo, &hi);
                int64_t deg = hi - lo;
                for (int32_t j = 0; j < nd; j++) {
                    uint64_t img = 0;
                    for (int32_t q = 0; q < nq; q++)
                        if (lm[j] >> q & 1) {
                            img |= succ[(int64_t)u * nq + q];
                            prod_edges += (int64_t)__builtin_popcountll(succ[(int64_t)u * nq + q]) * deg;
                        }
                    if (img) {
                        scans++;
                        scanned += deg;
                        bytes += 8 + (4 + word_bytes) * deg;
                    }
                }
            }
        }
        bytes += ((int64_t)nv + 7) / 8;
        counters[0] = prod_edges;
        counters[1] = scans;
        counters[2] = scanned;
        counters[3] = bytes;
        counters[4] = active;
        free(used); free(succ);
    }
    free(toff); free(tsym); free(ttgt);
    if (!dist_out) free(dist);
    return nlev;
}

/* The single-source query: og_ssr_from with V_s = {source}. */
int32_t og_ssr(const og_graph *g, int32_t nq, int32_t nfa_nl, const int64_t *sym_ptr,
               const int32_t *tfrom, const int32_t *tto, const int32_t *start, int32_t nstart,
               const int32_t *fin, int32_t nfin, int32_t source, uint64_t *bitmap,
               int32_t *dist_out, int64_t *level_counts, int32_t level_cap, int64_t *counters,
               int32_t word_bytes) {
    return og_ssr_from(g, nq, nfa_nl, sym_ptr, tfrom, tto, start, nstart, fin, nfin, &source, 1, bitmap,
                       dist_out, level_counts, level_cap, counters, word_bytes);
}
