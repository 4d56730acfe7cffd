// Stacked multi-source traversal (the multiple-source direction of Sec. 6):
// B sources under one NFA share one level-synchronous traversal. For every
// vertex v and state q, the frontier M and visited set P hold a row of B
// source bits (G = ceil(B/64) words), so the update of Alg. 1,
//     M' = ( OR over symbols a of (N^a)^T M G^a ) masked by not-P,   P = P + M',
// becomes, per edge (v, w) of symbol a and transition q -a-> q', an OR of the
// 64-bit words M[v][q][j] into w's row of q': one access to w's row serves 64
// sources per word (bit-parallel multi-source BFS, Then et al., VLDB 2014).
//
// The mask by not-P is deferred: an expansion ORs candidate bits into the next
// level's rows with fire-and-forget atomics (no read of P on the critical
// path of the scatter), and the next level's select applies the mask once
// per touched row while it builds the work items. On MI355X random 64-bit
// atomics cost more than twice a random load and never hit in L2, so this
// halves the atomics per edge against an atomic update of P.
//
// Phases per level (one cooperative launch, grid barriers between phases):
//   select  candidate vertex w -> masked frontier rows (P updated), frontier
//           state set S(w), and one item per used symbol u with
//           succ_u(S(w)) non-empty and a u-row at w;
//   push    (sparse levels) edges of all items spread evenly, G lanes per
//           edge (one source word each);
//   pull    (dense levels, at most 8 states) every row of the reverse
//           adjacency under a used symbol whose target states still miss
//           source bits gathers the frontier rows of its neighbours, stopping
//           once every bit is found; rows longer than PULL_LIGHT_ROW go to an
//           edge-balanced pass after a barrier.
// After the last level an extract phase turns the rows of final states into
// one result bitmap per source and resets P.
#include "../../include/rpq.h"
#include "device_common.h"
#include "stacked.h"

namespace rpq {

constexpr uint32_t PULL_LIGHT_ROW = 128;  // longer pull rows are processed edge-balanced
// Row lookups a select lane issues together: two keep the select phase
// kernel within 128 VGPRs (two workgroups per CU; with four it needs 141
// and gets one, and a large kg level's select took 4.9 ms instead of 3.0).
constexpr int ST_SYM_BATCH = 2;
// The expansion phase kernel: units per thread and step, threads per
// workgroup, and the waves per SIMD its registers are fitted to (none of
// these spill). More resident waves hide more of the gathers' and atomics'
// latency: on a large kg level (G = 4) the expansion took 14.5 ms at two
// 512-thread workgroups per CU with four units per thread, 12.5 ms at three
// with two units, and 11.2 ms at seven 256-thread workgroups with one unit
// (69 VGPRs; the 22.6 KB of LDS per workgroup allows seven).
template <int G>
constexpr int st_expand_upt() { return G <= 2 ? 2 : 1; }
template <int G>
constexpr int st_expand_threads() { return G <= 2 ? BLOCK : BLOCK / 2; }
template <int G>
constexpr int st_expand_waves() { return G <= 2 ? 6 : 7; }

// The query's tables for every phase of the stacked kernel: a copy in LDS
// when the block fits, else the global block.
__shared__ QueryView s_qv;
__shared__ __align__(16) uint8_t s_qc[QC_LDS_BYTES];

// Sets s_qv, copying the block into s_qc when it fits. Every thread of the
// workgroup calls it; it ends with a workgroup barrier.
__device__ __forceinline__ void st_qv_setup(const QueryView &qv) {
    const uint32_t nsym = qv.h->nsym;
    const size_t qb = qconst_bytes(nsym);
    const bool fits = qb <= QC_LDS_BYTES;
    if (fits) {
        const uint4 *src = reinterpret_cast<const uint4 *>(qv.h);
        uint4 *dst = reinterpret_cast<uint4 *>(s_qc);
        for (uint32_t i = threadIdx.x; i < (qb + 15) / 16; i += blockDim.x) dst[i] = src[i];
    }
    if (threadIdx.x == 0) s_qv = fits ? qconst_view(s_qc, nsym) : qv;
    __syncthreads();
}

__device__ __forceinline__ void sviol(const StackParams &p) { atomicAdd(&p.status[3], 1u); }

template <int G>
__device__ __forceinline__ uint64_t rowi(const StackParams &p, uint32_t v, uint32_t q) {
    return (static_cast<uint64_t>(v) * static_cast<uint32_t>(p.Q) + q) * G;
}

// The states of the automaton as a bit set (state sets read back from device
// memory are masked with it, so a row index never leaves its vertex).
__device__ __forceinline__ uint32_t state_mask(const StackParams &p) {
    return p.Q >= 32 ? ~0u : (1u << p.Q) - 1u;
}

// Queue length of record R, at most V (each vertex enters a queue once per
// level; a larger count is reported as a violated invariant).
__device__ __forceinline__ uint32_t queue_len(const StackParams &p, const LevelRec &R) {
    const uint32_t nq = ld_acq(&R.nq);
    const uint32_t V = static_cast<uint32_t>(p.V);
    if (nq > V) {
        if (gthread() == 0) sviol(p);
        return V;
    }
    return nq;
}

// Candidate and frontier state sets, one 32-bit word per vertex. (A byte per
// vertex for automata of up to 8 states was measured: 3 ms slower per kg
// launch, the atomics on words that four vertices share collide.)
template <int QM>
__device__ __forceinline__ uint32_t sup_ld(const uint32_t *a, uint32_t v) {
    return ldc(a + v);
}

template <int QM>
__device__ __forceinline__ void sup_st(uint32_t *a, uint32_t v, uint32_t x) {
    a[v] = x;
}

// OR x into v's set; returns the set before.
template <int QM>
__device__ __forceinline__ uint32_t sup_or(uint32_t *a, uint32_t v, uint32_t x) {
    return atomicOr(a + v, x);
}

// Bits of source word j that belong to real sources.
__device__ __forceinline__ uint64_t word_full(int32_t B, uint32_t j) {
    const int32_t r = B - 64 * static_cast<int32_t>(j);
    return r >= 64 ? ~0ull : r <= 0 ? 0ull : ((1ull << r) - 1ull);
}

// OR over the G consecutive lanes that work on one vertex (or edge). The
// lanes of a group always take the same branches, so they are active together.
template <int G>
__device__ __forceinline__ uint32_t group_or(uint32_t x) {
#pragma unroll
    for (int d = 1; d < G; d <<= 1) x |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(x), d, 64));
    return x;
}

template <int G>
__device__ __forceinline__ uint32_t group_sum(uint32_t x) {
#pragma unroll
    for (int d = 1; d < G; d <<= 1) x += static_cast<uint32_t>(__shfl_xor(static_cast<int>(x), d, 64));
    return x;
}

template <int G>
__device__ __forceinline__ uint64_t group_or64(uint64_t x) {
#pragma unroll
    for (int d = 1; d < G; d <<= 1) x |= __shfl_xor(x, d, 64);
    return x;
}

// LDS copy of the work items one workgroup is processing: at most CAP of
// them (a tile of TILE edges holds at most TILE / G + 1 items of G-word
// units; the persistent kernel keeps room for the G = 1 case).
template <uint32_t CAP>
struct StLdsN {
    static constexpr uint32_t cap = CAP;
    uint32_t eb[CAP], beg[CAP], v[CAP], u[CAP], s[CAP];
};
using StLds = StLdsN<TILE + 1>;

// Records item idx: `len` edges numbered from eb (both reserved by the caller
// with one atomic on a word that counts items in its high half and edges in
// its low half, so item order follows edge numbers), read from col[beg...].
// Every tile of TILE/G edges whose first edge the item holds points to it.
template <int G>
__device__ __forceinline__ void put_item(const StackParams &p, uint32_t idx, uint32_t eb, uint32_t beg, uint32_t len,
                                         uint32_t v, uint32_t u, uint32_t s) {
    constexpr uint32_t TE = TILE / G;
    if (idx < p.item_cap) {
        p.it_ebase[idx] = eb;
        p.it_beg[idx] = beg;
        p.it_v[idx] = v;
        p.it_u[idx] = u;
        p.it_s[idx] = s;
    } else {
        sviol(p);
    }
    const uint32_t k1 = (eb + len - 1) / TE;
    for (uint32_t k = (eb + TE - 1) / TE; k <= k1; k++) {
        if (k < p.tile_cap) p.tile_first[k] = idx;
        else { sviol(p); break; }
    }
}

// ------------------------------------------------------------------ select
// COUNT = false leaves out the work counters and the update count (a launch
// without RPQ_COUNTERS), which frees the registers they take.
template <int G, int QM, bool COUNT = true>
__device__ __forceinline__ void st_select(const StackParams &p, uint32_t n, uint32_t bid, uint32_t nblk, uint64_t &cacc) {
    const GraphView &g = p.g;
    const QueryView &qv = s_qv;
    LevelRec *rec = p.rec;
    LevelRec &R = rec[n % REC_RING];
    const uint32_t nq = queue_len(p, R);
    const uint32_t V = static_cast<uint32_t>(p.V);
    const uint32_t qmask = state_mask(p);
    if (bid == 0 && threadIdx.x == 0) {
        rec_clear(rec[(n + 1) % REC_RING]);
        if (n < LVL_COUNT_CAP) p.lvl[static_cast<uint64_t>(n) * LVL_STRIDE + 3] = wall_clock64();
    }
    const uint32_t lane = lane_id();
    const uint32_t j = lane % G;
    const uint32_t grp = lane / G;
    constexpr uint32_t GPB = BLOCK / G;  // vertices per workgroup and step
    uint32_t *sold = p.sup[(n + 1) & 1];
    // level n-1's frontier state sets live in the array level n's expansion
    // fills: clear them. Its frontier rows may stay: every bit in them is in
    // P already, so a later select masks them out (it rewrites every row it
    // reads), and the extract phase clears them with P.
    if (n >= 1) {
        const uint32_t nprev = queue_len(p, rec[(n - 1) % REC_RING]);
        const int32_t *qold = p.q[(n + 1) & 1];
        const uint32_t stride = nblk * BLOCK;
        for (uint32_t i0 = bid * BLOCK + threadIdx.x; i0 < nprev; i0 += 8 * stride) {
            uint32_t vv[8];
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const uint32_t i = i0 + k * stride;
                vv[k] = i < nprev ? static_cast<uint32_t>(ldc(&qold[i])) : 0u;
            }
#pragma unroll
            for (int k = 0; k < 8; k++) {
                if (i0 + k * stride >= nprev) continue;
                if (vv[k] < V) sup_st<QM>(sold, vv[k], 0u);
                else sviol(p);
            }
        }
    }
    const int32_t *qc = p.q[n & 1];
    uint64_t *Mc = p.M[n & 1];
    uint32_t *sc = p.sup[n & 1];
    const uint32_t nsym = qv.h->nsym;
    uint64_t pairs = 0, upd = 0, c_scans = 0, c_edges = 0, c_wb = 0, c_pe = 0;
    uint32_t nfront = 0, su = 0;
    const bool counters = COUNT && qv.h->counters != 0;
    // workgroup-uniform loop: item reservations are made per workgroup
    for (uint32_t bbase = bid * GPB; bbase < nq; bbase += nblk * GPB) {
        const uint32_t i = bbase + threadIdx.x / G;
        uint32_t w = 0, cs = 0;
        bool ok = false;
        if (i < nq) {
            w = static_cast<uint32_t>(ldc(&qc[i]));
            if (w < V) {
                cs = sup_ld<QM>(sc, w) & qmask;
                ok = true;
            } else {
                if (j == 0) sviol(p);
                w = 0;
            }
        }
        // mask the candidate rows by P (Alg. 1's complement mask), add the new
        // bits to P; rows that gained nothing are cleared
        uint32_t S = 0, nzm = 0, halves = 0;
        uint32_t pk[QM];  // new source bits per state in this lane's word (counters only)
#pragma unroll
        for (int k = 0; k < QM; k++) {
            pk[k] = 0;
            if ((cs >> k) & 1u) {
                const uint64_t idx = rowi<G>(p, w, k) + j;
                const uint64_t c = ldc(&Mc[idx]);
                const uint64_t pv = ldc(&p.P[idx]);
                const uint64_t nb = c & ~pv;
                if (nb) {
                    p.P[idx] = pv | nb;
                    nzm |= 1u << k;
                    pk[k] = static_cast<uint32_t>(__popcll(nb));
                    pairs += pk[k];
                    if constexpr (COUNT)
                        halves += (static_cast<uint32_t>(nb) != 0u) + (static_cast<uint32_t>(nb >> 32) != 0u);
                }
                if (nb != c) Mc[idx] = nb;
            }
        }
        S = group_or<G>(nzm);
        // work counters: W = 4 bytes per non-zero 32-bit word of the vertex's
        // frontier column (all states, all sources), and the frontier's pairs
        // per state over the group's words (for the product edges)
        uint32_t Wv = 0;
        if (counters) {
            Wv = 4u * group_sum<G>(halves);
#pragma unroll
            for (int k = 0; k < QM; k++) pk[k] = group_sum<G>(pk[k]);
            if (j == 0) c_wb += 2ull * Wv;
        }
        if (ok && j == 0) {
            sup_st<QM>(sc, w, S);
            if (S) nfront++;
            su |= S;
        }
        // nonzero source words per state over the group (for the work counter)
        uint32_t nzc[QM];
        if constexpr (COUNT) {
            const uint64_t gmask = ((1ull << G) - 1ull) << (grp * G);
#pragma unroll
            for (int k = 0; k < QM; k++) nzc[k] = static_cast<uint32_t>(__popcll(__ballot((nzm >> k) & 1u) & gmask));
        }
        // items: the small NFA factor first (succ_u of the state set), then
        // the neighbour range of the u-row at w. Only the symbols with a
        // transition out of S can give an item; lane j of the group looks up
        // and writes the items of the symbols u with u % G == j
        SymSet Rs = symbols_of(qv, S, nsym);
        {
            constexpr uint64_t PAT = G == 1 ? ~0ull
                                     : G == 2 ? 0x5555555555555555ull
                                     : G == 4 ? 0x1111111111111111ull
                                     : G == 8 ? 0x0101010101010101ull
                                              : 0x0001000100010001ull;
#pragma unroll
            for (int k = 0; k < SYM_WORDS; k++) Rs.w[k] &= PAT << j;
        }
        while (true) {
            uint32_t us[ST_SYM_BATCH], tu[ST_SYM_BATCH], beg[ST_SYM_BATCH], len[ST_SYM_BATCH];
            RankWordD rw[ST_SYM_BATCH];
#pragma unroll
            for (int jj = 0; jj < ST_SYM_BATCH; jj++) us[jj] = symbol_pop(Rs);
            bool more = false;
#pragma unroll
            for (int k = 0; k < SYM_WORDS; k++) more = more || Rs.w[k] != 0;
#pragma unroll
            for (int jj = 0; jj < ST_SYM_BATCH; jj++) {
                const uint32_t u = us[jj];
                tu[jj] = (S && u < nsym) ? succ_of(qv.succ, u, S) : 0u;
                if (tu[jj]) rw[jj] = g.rankw[qv.push_w[u] + (w >> 6)];
            }
            uint32_t cnt = 0, tot = 0;
#pragma unroll
            for (int jj = 0; jj < ST_SYM_BATCH; jj++) {
                const uint32_t u = us[jj];
                len[jj] = 0;
                uint32_t e;
                if constexpr (COUNT) c_scans += tu[jj] != 0u;
                if (tu[jj] && row_range(g, rw[jj], qv.push_r[u], w, beg[jj], e)) {
                    if (e > beg[jj] && e <= g.ncol) len[jj] = e - beg[jj];
                    else if (e != beg[jj]) sviol(p);
                }
                if (len[jj]) {
                    if constexpr (COUNT) {
                        // (edge, transition, word) updates this item carries
                        // and, with the counters, its product edges:
                        // |succ_u(q)| per pair (q, source) of the frontier,
                        // per edge
                        const uint32_t *su_tab = qv.succ + u * MAX_STATES;
                        uint32_t c = 0;
                        uint64_t pe = 0;
#pragma unroll
                        for (int k = 0; k < QM; k++) {
                            if ((S >> k) & 1u) {
                                const uint32_t ns = static_cast<uint32_t>(__popc(su_tab[k]));
                                c += ns * nzc[k];
                                pe += static_cast<uint64_t>(ns) * pk[k];
                            }
                        }
                        upd += static_cast<uint64_t>(c) * len[jj];
                        if (counters) {
                            c_pe += pe * len[jj];
                            c_wb += static_cast<uint64_t>(Wv) * len[jj];
                        }
                    }
                    cnt++;
                    tot += len[jj];
                }
            }
            uint64_t wtot;
            const uint64_t ex = wave_excl_scan((static_cast<uint64_t>(cnt) << 32) | tot, wtot);
            uint64_t wbase;
            const bool bmore = block_reserve<uint64_t>(wtot, more, &R.sel, wbase);
            if (cnt) {
                const uint64_t mine = wbase + ex;
                uint32_t idx = static_cast<uint32_t>(mine >> 32);
                uint32_t eb = static_cast<uint32_t>(mine);
                if constexpr (COUNT) c_edges += tot;
#pragma unroll
                for (int jj = 0; jj < ST_SYM_BATCH; jj++) {
                    if (!len[jj]) continue;
                    put_item<G>(p, idx, eb, beg[jj], len[jj], w, us[jj], S);
                    idx++;
                    eb += len[jj];
                }
            }
            if (!bmore) break;
        }
    }
    // level totals and work counters: one atomic per workgroup and field
    const uint64_t nf = wave_sum(nfront);
    const uint64_t v[3 + ST_NCNT] = {wave_sum(pairs),  nf,           wave_or(su),       wave_sum(c_scans),
                                     wave_sum(c_edges), wave_sum(upd), nf,               wave_sum(c_wb),
                                     wave_sum(c_pe)};
    const uint64_t t = block_reduce<3 + ST_NCNT>(v, 4u);
    if (t) {
        switch (threadIdx.x) {
            case 0: atomicAdd(reinterpret_cast<unsigned long long *>(&R.pairs), (unsigned long long)t); break;
            case 1: atomicAdd(&R.nfront, static_cast<uint32_t>(t)); break;
            case 2: atomicOr(&R.su, static_cast<uint32_t>(t)); break;
            // work counters: kept by threads 3..8 over the whole launch and
            // added to p.cnt once at its end (one line for all of them: per
            // level, the grid's atomics on it would queue for ~12 us)
            default:
                if (threadIdx.x < 3 + ST_NCNT) cacc += t;
                break;
        }
    }
}

// --------------------------------------------------------------- expansion
// One unit's state between its gather and its scatter.
template <int QM>
struct UnitC {
    uint64_t c[QM <= 8 ? QM : 1];  // new candidate bits per target state (QM <= 8)
    uint32_t dst;                  // target vertex (V when the unit is idle)
    uint32_t tb;                   // target states that received bits
};

// Gather of one unit: locate its item and edge, OR the source's frontier rows
// over the transitions into each target state, and drop the bits already in
// P. Wide automata (QM = 32) scatter here, one transition at a time.
// The staged item of each of K units: the last lo with L.eb[lo] <= the unit's
// edge. The halving steps depend on cnt alone (the same in every lane), so
// they run as one uniform loop of ceil(log2(cnt)) steps for all K units; a
// unit past uend searches for the range's last unit, and its caller drops it.
template <int G, int K, class LT>
__device__ __forceinline__ void item_search(const LT &L, uint32_t cnt, const uint64_t (&unit)[K], uint64_t uend,
                                            uint32_t (&lo)[K]) {
    uint32_t t[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        t[k] = static_cast<uint32_t>((unit[k] < uend ? unit[k] : uend - 1) / G);
        lo[k] = 0;
    }
    for (uint32_t len = __builtin_amdgcn_readfirstlane(cnt); len > 1;) {
        const uint32_t half = len >> 1;
#pragma unroll
        for (int k = 0; k < K; k++)
            if (L.eb[lo[k] + half] <= t[k]) lo[k] += half;
        len -= half;
    }
}

template <int G, int QM, bool PULL, class LT>
__device__ __forceinline__ void unit_gather(const StackParams &p, uint32_t n, const LT &L, uint32_t lo,
                                            uint64_t unit, uint64_t uend, uint32_t ns, UnitC<QM> &U) {
    const uint32_t V = static_cast<uint32_t>(p.V);
    const uint32_t j = static_cast<uint32_t>(unit % G);
    const uint64_t *Mc = p.M[n & 1];
    uint64_t *Mn = p.M[(n + 1) & 1];
    U.dst = V;
    U.tb = 0;
#pragma unroll
    for (int q2 = 0; q2 < (QM <= 8 ? QM : 1); q2++) U.c[q2] = 0;
    const uint32_t t = static_cast<uint32_t>(unit / G);
    // lo: the staged item holding edge t (item_search)
    if (unit >= uend) return;
    const uint32_t pos = L.beg[lo] + (t - L.eb[lo]);
    const uint32_t iv = L.v[lo], u = L.u[lo];
    if (pos >= p.g.ncol || iv >= V || u >= s_qv.h->nsym) {
        sviol(p);
        return;
    }
    const uint32_t other = p.g.col[pos];
    if (other >= V) {
        sviol(p);
        return;
    }
    const uint32_t src = PULL ? other : iv;
    const uint32_t w = PULL ? iv : other;
    const uint32_t *succ = s_qv.succ + u * MAX_STATES;
    const uint32_t tmask = PULL ? ns : ~0u;
    const uint32_t S = (PULL ? (sup_ld<QM>(p.sup[n & 1], src) & L.s[lo]) : L.s[lo]) & state_mask(p);
    U.dst = w;
    if constexpr (QM <= 8) {
        // y[q'] = OR of the source's rows over the transitions into q'
        uint64_t y[QM];
#pragma unroll
        for (int q2 = 0; q2 < QM; q2++) y[q2] = 0;
#pragma unroll
        for (int kq = 0; kq < QM; kq++) {
            if ((S >> kq) & 1u) {
                const uint64_t x = ldc(&Mc[rowi<G>(p, src, kq) + j]);
                const uint32_t tq = succ[kq] & tmask;
#pragma unroll
                for (int q2 = 0; q2 < QM; q2++)
                    if ((tq >> q2) & 1u) y[q2] |= x;
            }
        }
#pragma unroll
        for (int q2 = 0; q2 < QM; q2++)
            if (y[q2]) U.c[q2] = y[q2] & ~ldc(&p.P[rowi<G>(p, w, q2) + j]);
    } else {
        uint32_t SS = S;
        while (SS) {
            const uint32_t kq = __ffs(SS) - 1;
            SS &= SS - 1;
            uint32_t tq = succ[kq] & tmask;
            if (!tq) continue;
            const uint64_t x = ldc(&Mc[rowi<G>(p, src, kq) + j]);
            if (!x) continue;
            while (tq) {
                const uint32_t q2 = __ffs(tq) - 1;
                tq &= tq - 1;
                const uint64_t idx = rowi<G>(p, w, q2) + j;
                const uint64_t c = x & ~ldc(&p.P[idx]);
                if (c) {
                    atomicOr(reinterpret_cast<unsigned long long *>(Mn + idx), static_cast<unsigned long long>(c));
                    U.tb |= 1u << q2;
                }
            }
        }
    }
}

// Scatter of one unit (QM <= 8): fire-and-forget ORs into the target's rows.
template <int G, int QM>
__device__ __forceinline__ void unit_scatter(const StackParams &p, uint32_t n, uint32_t j, UnitC<QM> &U) {
    if constexpr (QM <= 8) {
        uint64_t *Mn = p.M[(n + 1) & 1];
#pragma unroll
        for (int q2 = 0; q2 < QM; q2++) {
            if (U.c[q2]) {
                atomicOr(reinterpret_cast<unsigned long long *>(Mn + rowi<G>(p, U.dst, q2) + j),
                         static_cast<unsigned long long>(U.c[q2]));
                U.tb |= 1u << q2;
            }
        }
    }
}

// The first writer of the target's candidate state set appends it to the
// next queue. Every thread of the workgroup calls this.
template <int G, int QM>
__device__ __forceinline__ void unit_append(const StackParams &p, uint32_t n, uint32_t j, const UnitC<QM> &U) {
    const uint32_t tg = group_or<G>(U.tb);
    bool first = false;
    if (tg && j == 0) first = sup_or<QM>(p.sup[(n + 1) & 1], U.dst, tg) == 0u;
    if (!block_append(first, static_cast<int32_t>(U.dst), p.q[(n + 1) & 1], &p.rec[(n + 1) % REC_RING].nq,
                      static_cast<uint32_t>(p.V)))
        sviol(p);
}

// Four units' appends with their sup atomics issued together and one queue
// reservation per workgroup. Every thread of the workgroup calls this.
template <int G, int QM>
__device__ __forceinline__ void unit_append4(const StackParams &p, uint32_t n, uint32_t j, const UnitC<QM> &U0,
                                             const UnitC<QM> &U1, const UnitC<QM> &U2, const UnitC<QM> &U3) {
    uint32_t *sn = p.sup[(n + 1) & 1];
    const uint32_t t0 = group_or<G>(U0.tb), t1 = group_or<G>(U1.tb);
    const uint32_t t2 = group_or<G>(U2.tb), t3 = group_or<G>(U3.tb);
    const bool lead = j == 0;
    // a plain load first: on dense levels most targets already hold the
    // states (values read during the phase only ever lack bits, never have
    // extra ones), and a load costs far less than an atomic
    uint32_t o0 = 1, o1 = 1, o2 = 1, o3 = 1;
    if (t0 && lead) o0 = sup_ld<QM>(sn, U0.dst);
    if (t1 && lead) o1 = sup_ld<QM>(sn, U1.dst);
    if (t2 && lead) o2 = sup_ld<QM>(sn, U2.dst);
    if (t3 && lead) o3 = sup_ld<QM>(sn, U3.dst);
    if (t0 && lead && (o0 & t0) != t0) o0 = sup_or<QM>(sn, U0.dst, t0);
    if (t1 && lead && (o1 & t1) != t1) o1 = sup_or<QM>(sn, U1.dst, t1);
    if (t2 && lead && (o2 & t2) != t2) o2 = sup_or<QM>(sn, U2.dst, t2);
    if (t3 && lead && (o3 & t3) != t3) o3 = sup_or<QM>(sn, U3.dst, t3);
    if (!block_append4(o0 == 0, static_cast<int32_t>(U0.dst), o1 == 0, static_cast<int32_t>(U1.dst), o2 == 0,
                       static_cast<int32_t>(U2.dst), o3 == 0, static_cast<int32_t>(U3.dst), p.q[(n + 1) & 1],
                       &p.rec[(n + 1) % REC_RING].nq, static_cast<uint32_t>(p.V)))
        sviol(p);
}

// Dense levels: the target's candidate state set only (no queue append; the
// queue is built afterwards by st_compact, in vertex order). A plain load
// first, as in unit_append4; the OR needs no return value.
template <int G, int QM>
__device__ __forceinline__ void unit_mark(const StackParams &p, uint32_t n, uint32_t j, const UnitC<QM> &U) {
    const uint32_t t = group_or<G>(U.tb);
    if (t && j == 0) {
        uint32_t *sn = p.sup[(n + 1) & 1];
        if ((sup_ld<QM>(sn, U.dst) & t) != t) (void)sup_or<QM>(sn, U.dst, t);
    }
}

template <int G, int QM>
__device__ __forceinline__ void unit_mark4(const StackParams &p, uint32_t n, uint32_t j, const UnitC<QM> &U0,
                                           const UnitC<QM> &U1, const UnitC<QM> &U2, const UnitC<QM> &U3) {
    uint32_t *sn = p.sup[(n + 1) & 1];
    const uint32_t t0 = group_or<G>(U0.tb), t1 = group_or<G>(U1.tb);
    const uint32_t t2 = group_or<G>(U2.tb), t3 = group_or<G>(U3.tb);
    if (j != 0) return;
    uint32_t o0 = ~0u, o1 = ~0u, o2 = ~0u, o3 = ~0u;
    if (t0) o0 = sup_ld<QM>(sn, U0.dst);
    if (t1) o1 = sup_ld<QM>(sn, U1.dst);
    if (t2) o2 = sup_ld<QM>(sn, U2.dst);
    if (t3) o3 = sup_ld<QM>(sn, U3.dst);
    if ((o0 & t0) != t0) (void)sup_or<QM>(sn, U0.dst, t0);
    if ((o1 & t1) != t1) (void)sup_or<QM>(sn, U1.dst, t1);
    if ((o2 & t2) != t2) (void)sup_or<QM>(sn, U2.dst, t2);
    if ((o3 & t3) != t3) (void)sup_or<QM>(sn, U3.dst, t3);
}

// Level n+1's queue from its candidate state sets, in vertex order: every
// workgroup takes a contiguous range of vertices, 8 per thread and step, and
// reserves its step's queue positions with one atomic. Follows an expansion
// that marked the sets only (unit_mark4); the next select then reads rows,
// state sets and rank words of consecutive vertices.
__device__ __forceinline__ void st_compact(const StackParams &p, uint32_t n) {
    constexpr uint32_t PER = 8;
    constexpr uint32_t STEP = BLOCK * PER;
    const uint32_t V = static_cast<uint32_t>(p.V);
    const uint32_t *sn = p.sup[(n + 1) & 1];
    int32_t *qn = p.q[(n + 1) & 1];
    uint32_t *cnt = &p.rec[(n + 1) % REC_RING].nq;
    const uint32_t per_wg = (V + gridDim.x - 1) / gridDim.x;
    const uint32_t chunk = (per_wg + STEP - 1) / STEP * STEP;
    const uint64_t c0 = static_cast<uint64_t>(blockIdx.x) * chunk;
    const uint64_t c1 = c0 + chunk < V ? c0 + chunk : V;
    for (uint64_t b = c0; b < c1; b += STEP) {  // workgroup-uniform
        const uint64_t v0 = b + static_cast<uint64_t>(threadIdx.x) * PER;
        uint32_t m = 0;
#pragma unroll
        for (uint32_t k = 0; k < PER; k++)
            if (v0 + k < c1 && ldc(&sn[v0 + k]) != 0u) m |= 1u << k;
        uint64_t wtot;
        const uint64_t ex = wave_excl_scan(static_cast<uint64_t>(__popc(m)), wtot);
        uint32_t wbase = 0;
        block_reserve<uint32_t>(static_cast<uint32_t>(wtot), false, cnt, wbase);
        uint32_t pos = wbase + static_cast<uint32_t>(ex);
        while (m) {
            const uint32_t k = __ffs(m) - 1;
            m &= m - 1;
            if (pos < V) qn[pos] = static_cast<int32_t>(v0 + k);
            else sviol(p);
            pos++;
        }
    }
}

// Edge-balanced pull of long rows: when every lane of the wave works on the
// same target row, OR the candidate words of each source word j over the
// wave and leave them in lanes 0..G-1, so a hub's row costs one atomic per
// (state, word) and wave instead of one per edge.
template <int G, int QM>
__device__ __forceinline__ void wave_merge(UnitC<QM> &U) {
    const uint32_t d0 = static_cast<uint32_t>(__shfl(static_cast<int>(U.dst), 0, 64));
    if (__ballot(U.dst != d0) != 0) return;
#pragma unroll
    for (int q2 = 0; q2 < QM; q2++) {
        uint64_t c = U.c[q2];
#pragma unroll
        for (int d = G; d < 64; d <<= 1) c |= __shfl_xor(c, d, 64);
        U.c[q2] = lane_id() < static_cast<uint32_t>(G) ? c : 0ull;
    }
}

// Units [ubase, uend) of the items staged in L (cnt of them): unit t*G + j is
// source word j of the level's edge number t. Push: the item is (v, u) and the
// edge leads to w; the frontier rows of v are ORed into w's candidate rows.
// Pull (long rows): the item is (w, u) with the reverse neighbour v on the
// edge; only states in sup[v] & L.s (predecessors of the wanted states) count.
// Either way the candidate bits already in P are dropped before the atomic
// OR, and the first writer of sup_next[w] appends w to the next queue. UPT
// units per thread are gathered before any is scattered (QM <= 8), so their
// loads overlap; fewer units per thread take fewer registers and leave room
// for more waves.
template <int G, int QM, bool PULL, bool MARK, int UPT, int NT, class LT>
__device__ __forceinline__ void expand_range(const StackParams &p, uint32_t n, const LT &L, uint32_t cnt, uint64_t ubase,
                                             uint64_t uend, uint32_t ns) {
    const uint32_t tid = threadIdx.x;
    const uint32_t j = tid % G;
    if constexpr (QM <= 8) {
        static_assert(TILE % (UPT * NT) == 0, "a tile is whole steps of the workgroup");
        for (uint64_t ub = ubase; ub < uend; ub += UPT * NT) {
            UnitC<QM> U[UPT];
            uint64_t us[UPT];
#pragma unroll
            for (int k = 0; k < UPT; k++) us[k] = ub + static_cast<uint64_t>(k) * NT + tid;
            uint32_t lo[UPT];
            item_search<G, UPT>(L, cnt, us, uend, lo);
#pragma unroll
            for (int k = 0; k < UPT; k++) unit_gather<G, QM, PULL>(p, n, L, lo[k], us[k], uend, ns, U[k]);
            if constexpr (PULL) {
#pragma unroll
                for (int k = 0; k < UPT; k++) wave_merge<G, QM>(U[k]);
            }
#pragma unroll
            for (int k = 0; k < UPT; k++) unit_scatter<G, QM>(p, n, j, U[k]);
            if constexpr (UPT == 4) {
                if constexpr (MARK) unit_mark4<G, QM>(p, n, j, U[0], U[1], U[2], U[3]);
                else unit_append4<G, QM>(p, n, j, U[0], U[1], U[2], U[3]);
            } else {
#pragma unroll
                for (int k = 0; k < UPT; k++) {
                    if constexpr (MARK) unit_mark<G, QM>(p, n, j, U[k]);
                    else unit_append<G, QM>(p, n, j, U[k]);
                }
            }
        }
    } else {
        for (uint64_t ub = ubase; ub < uend; ub += NT) {
            UnitC<QM> U0;
            const uint64_t us[1] = {ub + tid};
            uint32_t lo[1];
            item_search<G, 1>(L, cnt, us, uend, lo);
            unit_gather<G, QM, PULL>(p, n, L, lo[0], us[0], uend, ns, U0);
            if constexpr (MARK) unit_mark<G, QM>(p, n, j, U0);
            else unit_append<G, QM>(p, n, j, U0);
        }
    }
}

// Items [0, nitems) with `T` edges (packed in sel) -> units spread over the grid.
template <int G, int QM, bool PULL, bool MARK = false, int UPT = 4, int NT = BLOCK, class LT = StLds>
__device__ __forceinline__ void expand_items(const StackParams &p, uint32_t n, LT &L, uint64_t sel, uint32_t ns,
                                             uint32_t bid, uint32_t nblk) {
    constexpr uint32_t TE = TILE / G;
    static_assert(LT::cap >= TE + 1, "room for the items of one tile");
    const uint32_t nitems = static_cast<uint32_t>(sel >> 32);
    const uint32_t T = static_cast<uint32_t>(sel);
    if (T == 0 || nitems == 0) return;
    if (nitems > p.item_cap) {
        if (bid == 0 && threadIdx.x == 0) sviol(p);
        return;
    }
    const uint64_t units = static_cast<uint64_t>(T) * G;
    const uint32_t tid = threadIdx.x;
    if (nitems < LT::cap) {
        // few items: every workgroup stages all of them and takes an even,
        // wave-aligned share of the units, so small levels use the whole chip
        for (uint32_t x = tid; x < nitems; x += NT) {
            L.eb[x] = ldc(&p.it_ebase[x]);
            L.beg[x] = ldc(&p.it_beg[x]);
            L.v[x] = ldc(&p.it_v[x]);
            L.u[x] = ldc(&p.it_u[x]);
            L.s[x] = ldc(&p.it_s[x]);
        }
        __syncthreads();
        uint64_t per = (units + nblk - 1) / nblk;
        per = (per + 63) & ~63ull;
        const uint64_t b0 = static_cast<uint64_t>(bid) * per;
        const uint64_t b1 = b0 + per < units ? b0 + per : units;
        if (b0 < b1) expand_range<G, QM, PULL, MARK, UPT, NT>(p, n, L, nitems, b0, b1, ns);
        __syncthreads();
        return;
    }
    const uint32_t ntiles = (T + TE - 1) / TE;
    // fewer tiles than workgroups: split each tile into parts of at least a
    // wave's worth of units, so the level still spreads over the grid
    uint32_t sub = 1;
    while (sub < TILE / 64 && ntiles * sub * 2 <= nblk) sub *= 2;
    const uint32_t part_units = TILE / sub;
    for (uint32_t vt = bid; vt < ntiles * sub; vt += nblk) {
        const uint32_t tile = vt / sub, part = vt % sub;
        uint32_t i0 = tile < p.tile_cap ? ldc(&p.tile_first[tile]) : 0u;
        uint32_t i1 = (tile + 1 < ntiles && tile + 1 < p.tile_cap) ? ldc(&p.tile_first[tile + 1]) : nitems - 1;
        if (i0 >= nitems || i1 >= nitems || i1 < i0 || i1 - i0 > TE) {
            if (tid == 0) sviol(p);
            i0 = i1 = 0;
        }
        const uint32_t cnt = i1 - i0 + 1;
        for (uint32_t x = tid; x < cnt; x += NT) {
            L.eb[x] = ldc(&p.it_ebase[i0 + x]);
            L.beg[x] = ldc(&p.it_beg[i0 + x]);
            L.v[x] = ldc(&p.it_v[i0 + x]);
            L.u[x] = ldc(&p.it_u[i0 + x]);
            L.s[x] = ldc(&p.it_s[i0 + x]);
        }
        __syncthreads();
        const uint64_t u0 = static_cast<uint64_t>(tile) * TILE + static_cast<uint64_t>(part) * part_units;
        const uint64_t u1 = u0 + part_units < units ? u0 + part_units : units;
        if (u0 < u1) expand_range<G, QM, PULL, MARK, UPT, NT>(p, n, L, cnt, u0, u1, ns);
        __syncthreads();
    }
}

// Dense levels (at most 8 states), row by row: for every used symbol u that
// leads into the states `ns` the level can produce, every row of u's pull
// direction (a vertex w with reverse u-neighbours; rows are stored in vertex
// order with their vertex ids, so no lookup is needed) whose target states
// still miss source bits gathers the frontier rows of its neighbours (4 in
// flight) and stops as soon as every missing bit is found. One atomic OR per
// (row, target state, word) carries the result. Rows longer than
// PULL_LIGHT_ROW become items of the edge-balanced pass.
template <int G>
__device__ __forceinline__ void st_pull_rows(const StackParams &p, uint32_t n, uint32_t ns) {
    const GraphView &g = p.g;
    const QueryView &qv = s_qv;
    const uint32_t V = static_cast<uint32_t>(p.V);
    const uint32_t nsym = qv.h->nsym;
    const uint32_t lane = lane_id();
    const uint32_t j = lane % G;
    constexpr uint32_t GPB = BLOCK / G;  // rows per workgroup and step
    const uint64_t full = word_full(p.B, j);
    const uint64_t *Mc = p.M[n & 1];
    uint64_t *Mn = p.M[(n + 1) & 1];
    const uint32_t *sc = p.sup[n & 1];
    uint32_t *sn = p.sup[(n + 1) & 1];
    int32_t *qn = p.q[(n + 1) & 1];
    LevelRec &R = p.rec[n % REC_RING];
    LevelRec &RN = p.rec[(n + 1) % REC_RING];
    for (uint32_t u = 0; u < nsym; u++) {
        const uint32_t *pred = qv.pred + u * MAX_STATES;
        const uint32_t *succ = qv.succ + u * MAX_STATES;
        // states that reach `ns` over u, and the states they reach
        uint32_t pu = 0, x = ns;
        while (x) {
            pu |= pred[__ffs(x) - 1];
            x &= x - 1;
        }
        uint32_t tu = 0;
        x = pu;
        while (x) {
            tu |= succ[__ffs(x) - 1];
            x &= x - 1;
        }
        tu &= ns;
        if (!pu || !tu) continue;
        const uint64_t rb = qv.pull_r[u];
        const uint32_t rows = qv.pull_n[u];
        // workgroup-uniform loop: reservations are made per workgroup
        for (uint32_t bbase = blockIdx.x * GPB; bbase < rows; bbase += gridDim.x * GPB) {
            const uint32_t r = bbase + threadIdx.x / G;
            uint32_t w = V, beg = 0, end = 0;
            if (r < rows) {
                w = g.rowvert[rb + r];
                beg = g.rowptr[rb + r];
                end = g.rowptr[rb + r + 1];
                if (w >= V || end > g.ncol || end < beg) {
                    if (j == 0) sviol(p);
                    w = V;
                }
            }
            uint64_t prow[8], acc[8];
            uint64_t need = 0;
#pragma unroll
            for (int k = 0; k < 8; k++) {
                prow[k] = 0;
                acc[k] = 0;
                if (w < V && ((tu >> k) & 1u)) {
                    prow[k] = ldc(&p.P[rowi<G>(p, w, k) + j]);
                    need |= full & ~prow[k];
                }
            }
            need = group_or64<G>(need);
            uint32_t tb = 0;
            bool heavy = false;
            if (need) {
                if (end - beg > PULL_LIGHT_ROW) {
                    heavy = true;
                } else {
                    for (uint32_t e0 = beg; e0 < end && need; e0 += 4) {
                        uint32_t vv[4], sv[4];
#pragma unroll
                        for (int a = 0; a < 4; a++) vv[a] = e0 + a < end ? g.col[e0 + a] : V;
#pragma unroll
                        for (int a = 0; a < 4; a++) sv[a] = vv[a] < V ? (sup_ld<8>(sc, vv[a]) & pu) : 0u;  // pu: states only
#pragma unroll
                        for (int a = 0; a < 4; a++) {
#pragma unroll
                            for (int kq = 0; kq < 8; kq++) {
                                if ((sv[a] >> kq) & 1u) {
                                    const uint64_t xw = ldc(&Mc[rowi<G>(p, vv[a], kq) + j]);
                                    const uint32_t tq = succ[kq] & tu;
#pragma unroll
                                    for (int k2 = 0; k2 < 8; k2++)
                                        if ((tq >> k2) & 1u) acc[k2] |= xw;
                                }
                            }
                        }
                        uint64_t rem = 0;
#pragma unroll
                        for (int k = 0; k < 8; k++)
                            if ((tu >> k) & 1u) rem |= full & ~(prow[k] | acc[k]);
                        need = group_or64<G>(rem);
                    }
#pragma unroll
                    for (int k = 0; k < 8; k++) {
                        const uint64_t m = acc[k] & ~prow[k];
                        if (m) {
                            atomicOr(reinterpret_cast<unsigned long long *>(Mn + rowi<G>(p, w, k) + j),
                                     static_cast<unsigned long long>(m));
                            tb |= 1u << k;
                        }
                    }
                }
            }
            // long rows become items of the edge-balanced pass; rows that
            // gained bits are appended to the next queue (the first writer of
            // their state set): both reserved together, once per workgroup
            const bool hl = heavy && j == 0;
            uint64_t htot;
            const uint64_t hex =
                wave_excl_scan(hl ? ((1ull << 32) | static_cast<uint64_t>(end - beg)) : 0ull, htot);
            tb = group_or<G>(tb);
            bool first = false;
            if (tb && j == 0) first = sup_or<8>(sn, w, tb) == 0u;
            const uint64_t fm = __ballot(first);
            uint64_t hbase;
            uint32_t qbase;
            block_reserve2(htot, &R.hsel, hbase, static_cast<uint32_t>(__popcll(fm)), &RN.nq, qbase);
            if (hl) {
                const uint64_t at = hbase + hex;
                put_item<G>(p, static_cast<uint32_t>(at >> 32), static_cast<uint32_t>(at), beg, end - beg, w, u, pu);
            }
            if (first) {
                const uint32_t pos = qbase + static_cast<uint32_t>(__popcll(fm & ((1ull << lane) - 1ull)));
                if (pos < V) qn[pos] = static_cast<int32_t>(w);
                else sviol(p);
            }
        }
    }
}

// ------------------------------------------------------------- direction
// push (0) or pull (1) for level n; every workgroup computes the same answer
template <int QM>
__device__ __forceinline__ uint32_t st_decide(const StackParams &p, uint32_t n, uint32_t prev) {
    const QHeader &h = *s_qv.h;
    if (QM > 8 || h.force == 1) return 0;
    if (h.force == 2) return 1;
    if (!(h.alpha > 0.f)) return 0;
    const LevelRec &R = p.rec[n % REC_RING];
    const uint64_t T = ld_acq(&R.sel) & 0xffffffffull;
    if (prev == 0) return static_cast<double>(T) * h.alpha > static_cast<double>(h.e_rel) ? 1u : 0u;
    const uint32_t nf = ld_acq(&R.nfront);
    return static_cast<double>(nf) * h.beta < static_cast<double>(p.V) ? 0u : 1u;
}

// --------------------------------------------------------------- extract
// Result: source b reaches v iff some final state's row at v has bit b. A
// wavefront holds 64 consecutive vertices, one per lane, and 64 ballots
// transpose each source word of the block into one output word per source.
// P and the last frontier are reset.
template <int G, int QM>
__device__ __forceinline__ void st_final(const StackParams &p, uint32_t nexit, uint32_t levels) {
    const uint32_t V = static_cast<uint32_t>(p.V);
    const uint32_t Q = static_cast<uint32_t>(p.Q);
    if (blockIdx.x == 0 && threadIdx.x == 0 && levels < LVL_COUNT_CAP)
        p.lvl[static_cast<uint64_t>(levels) * LVL_STRIDE + 3] = wall_clock64();
    const uint32_t lane = lane_id();
    // the last frontier's state sets, then both row buffers (rows keep
    // visited bits between levels; see the select phase)
    if (nexit >= 1) {
        const uint32_t D = nexit - 1;
        const uint32_t nq = queue_len(p, p.rec[D % REC_RING]);
        uint32_t *sp = p.sup[D & 1];
        const int32_t *q = p.q[D & 1];
        for (uint32_t i = gthread(); i < nq; i += gthreads()) {
            const uint32_t v = static_cast<uint32_t>(ldc(&q[i]));
            if (v < V) sup_st<QM>(sp, v, 0u);
            else sviol(p);
        }
    }
    // Row words of M are cleared below with P's: every bit an expansion ORs
    // into M is added to P by the next select (or was there already), so M
    // is zero wherever P is.
    const uint32_t fm = s_qv.h->fmask;
    const uint64_t nwords = static_cast<uint64_t>(p.nwords);
    const uint64_t total = nwords * G;
    const uint32_t B = static_cast<uint32_t>(p.B);
    // With a probe vertex only its final-state rows are read, by workgroup
    // 0 (which also clears them; the loop below clears every other row).
    const bool probing = p.probe < V;
    if (probing && blockIdx.x == 0 && threadIdx.x < static_cast<uint32_t>(G)) {
        uint64_t f = 0;
        for (uint32_t q = 0; q < Q; q++) {
            const uint64_t idx = rowi<G>(p, p.probe, q) + threadIdx.x;
            const uint64_t x = ldc(&p.P[idx]);
            if (x) {
                if (fm >> q & 1u) f |= x;
                p.P[idx] = 0;
                p.M[0][idx] = 0;
                p.M[1][idx] = 0;
            }
        }
        p.out[threadIdx.x] = f & word_full(p.B, threadIdx.x);
    }
    if constexpr (G <= 4) {
        // A wave takes KC consecutive 64-vertex blocks. The rows of a block
        // are one contiguous range of P, read 64 consecutive words per load
        // (four whole lines, where a load of one word per vertex touches 64
        // lines); set words are cleared with the same pattern, and the
        // words of final states are ORed into the wave's LDS columns F[j],
        // one word per vertex. Lane l then holds vertex l's result words,
        // and 64 ballots per word j transpose them into one output word per
        // source; lane i stores KC consecutive words of source j*64 + i.
        constexpr uint32_t KC = 16 / G;
        __shared__ uint64_t s_f[BLOCK / 64][G][64];
        uint64_t(*F)[64] = s_f[threadIdx.x >> 6];
        const uint32_t QG = Q * G;
        const uint64_t nchunks = (nwords + KC - 1) / KC;
        for (uint64_t c = gthread() >> 6; c < nchunks; c += gthreads() >> 6) {  // wave-uniform
            uint64_t mine[G][KC];
#pragma unroll
            for (uint32_t kk = 0; kk < KC; kk++) {
                const uint64_t v0 = (c * KC + kk) * 64;
#pragma unroll
                for (int j = 0; j < G; j++) F[j][lane] = 0;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if (v0 < V) {
                    const uint32_t nv = V - v0 < 64 ? static_cast<uint32_t>(V - v0) : 64u;
                    const uint32_t words = nv * QG;
                    const uint64_t base = v0 * QG;  // rowi(v0, 0)
                    for (uint32_t i0 = 0; i0 < words; i0 += 4 * 64) {
                        uint64_t x[4];
#pragma unroll
                        for (uint32_t r = 0; r < 4; r++) {
                            const uint32_t i = i0 + r * 64 + lane;
                            x[r] = i < words ? ldc(&p.P[base + i]) : 0ull;
                        }
#pragma unroll
                        for (uint32_t r = 0; r < 4; r++) {
                            if (!x[r]) continue;
                            const uint32_t i = i0 + r * 64 + lane;
                            const uint32_t vl = i / QG;
                            const uint32_t rem = i - vl * QG;
                            if (probing && v0 + vl == p.probe) continue;
                            p.P[base + i] = 0;
                            p.M[0][base + i] = 0;
                            p.M[1][base + i] = 0;
                            if (fm >> (rem / G) & 1u)
                                atomicOr(reinterpret_cast<unsigned long long *>(&F[rem % G][vl]),
                                         static_cast<unsigned long long>(x[r]));
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
                for (int j = 0; j < G; j++) {
                    const uint64_t f = F[j][lane];
                    uint64_t t = 0;
                    if (!probing) {  // uniform: the probe is a launch parameter
                        for (uint32_t i = 0; i < 64; i++) {
                            const uint64_t bl = __ballot((f >> i) & 1ull);
                            if (lane == i) t = bl;
                        }
                    }
                    mine[j][kk] = t;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // F is read before the next block clears it
            }
            if (probing) continue;
#pragma unroll
            for (int j = 0; j < G; j++) {
                const uint32_t src = j * 64 + lane;
                if (src >= B) continue;
#pragma unroll
                for (uint32_t kk = 0; kk < KC; kk++) {
                    const uint64_t k = c * KC + kk;
                    if (k < nwords) p.out[static_cast<uint64_t>(src) * nwords + k] = mine[j][kk];
                }
            }
        }
        return;
    }
    if constexpr (QM * G <= 32) {
        // a wave takes KC consecutive 64-vertex blocks and every source word
        // of them: each lane loads its vertex's whole row (all loads in
        // flight together), and lane i of the wave then stores KC
        // consecutive output words of source j*64 + i for every word j
        constexpr uint32_t NW = QM * G;
        constexpr uint32_t KC = 16 / G;
        const uint32_t QG = Q * G;
        const uint64_t nchunks = (nwords + KC - 1) / KC;
        for (uint64_t c = gthread() >> 6; c < nchunks; c += gthreads() >> 6) {
            uint64_t mine[G][KC];
#pragma unroll
            for (uint32_t kk = 0; kk < KC; kk++) {
                const uint64_t k = c * KC + kk;
                const uint64_t v = k * 64 + lane;
                uint64_t f[G];
#pragma unroll
                for (int j = 0; j < G; j++) f[j] = 0;
                if (v < V && !(probing && v == p.probe)) {
                    const uint64_t r0 = rowi<G>(p, static_cast<uint32_t>(v), 0);
                    uint64_t x[NW];
#pragma unroll
                    for (uint32_t w = 0; w < NW; w++) x[w] = w < QG ? ldc(&p.P[r0 + w]) : 0ull;
#pragma unroll
                    for (uint32_t w = 0; w < NW; w++) {
                        if (x[w]) {
                            if (fm >> (w / G) & 1u) f[w % G] |= x[w];
                            p.P[r0 + w] = 0;
                            p.M[0][r0 + w] = 0;
                            p.M[1][r0 + w] = 0;
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < G; j++) {
                    uint64_t t = 0;
                    if (!probing) {  // uniform: the probe is a launch parameter
                        for (uint32_t i = 0; i < 64; i++) {
                            const uint64_t bl = __ballot((f[j] >> i) & 1ull);
                            if (lane == i) t = bl;
                        }
                    }
                    mine[j][kk] = t;
                }
            }
            if (probing) continue;
#pragma unroll
            for (int j = 0; j < G; j++) {
                const uint32_t src = j * 64 + lane;
                if (src >= B) continue;
#pragma unroll
                for (uint32_t kk = 0; kk < KC; kk++) {
                    const uint64_t k = c * KC + kk;
                    if (k < nwords) p.out[static_cast<uint64_t>(src) * nwords + k] = mine[j][kk];
                }
            }
        }
        return;
    }
    for (uint64_t gw = gthread() >> 6; gw < total; gw += gthreads() >> 6) {
        const uint64_t k = gw / G;
        const uint32_t j = static_cast<uint32_t>(gw % G);
        const uint64_t v = k * 64 + lane;
        uint64_t f = 0;
        if (v < V && !(probing && v == p.probe)) {
            const uint64_t r0 = rowi<G>(p, static_cast<uint32_t>(v), 0) + j;
            for (uint32_t q = 0; q < Q; q++) {
                const uint64_t x = ldc(&p.P[r0 + q * G]);
                if (x) {
                    if (fm >> q & 1u) f |= x;
                    p.P[r0 + q * G] = 0;
                    p.M[0][r0 + q * G] = 0;
                    p.M[1][r0 + q * G] = 0;
                }
            }
        }
        if (probing) continue;  // uniform: the probe is a launch parameter
        // transpose: lane i keeps the word of source j*64 + i (bit l = vertex
        // 64k + l) and the wave stores all of them with one instruction
        uint64_t mine = 0;
        for (uint32_t i = 0; i < 64; i++) {
            const uint64_t b = __ballot((f >> i) & 1ull);
            if (lane == i) mine = b;
        }
        const uint32_t src = j * 64 + lane;
        if (src < B) p.out[static_cast<uint64_t>(src) * nwords + k] = mine;
    }
}

// ----------------------------------------------------------------- kernel
// Level n's record once its select phase is complete (one thread).
__device__ __forceinline__ void st_record(const StackParams &p, uint32_t n, uint32_t mode) {
    LevelRec &R = p.rec[n % REC_RING];
    R.mode = mode;
    if (n < LVL_COUNT_CAP) {
        uint64_t *Lv = p.lvl + static_cast<uint64_t>(n) * LVL_STRIDE;
        Lv[0] = ld_acq(&R.pairs);
        Lv[1] = ld_acq(&R.nfront);
        Lv[2] = ld_acq(&R.sel);
        Lv[4] = wall_clock64();
    }
}

// ------------------------------------------------------------ small levels
// As in the single-query kernel: levels with a short candidate queue and few
// expansion units run in workgroup 0 alone, with workgroup barriers in place
// of grid barriers, while the other workgroups wait at one grid barrier.
constexpr uint32_t ST_SOLO_MAX_UNITS = 4 * TILE;  // expansion units of a small level
constexpr uint32_t ST_SOLO_MAX_RUN = 2048;        // levels per run (the waiting barrier times out after 5 s)

__device__ __forceinline__ void st_solo_sync() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Runs levels n, n+1, ... in workgroup 0 while they are small (one select
// step of the workgroup). Leaves in bar->solo_n the first level not
// finished and in bar->solo_sel whether its select phase is already done.
template <int G, int QM>
__device__ __forceinline__ void st_solo_levels(const StackParams &p, uint32_t n, StLds &L, uint32_t prev,
                                               uint32_t &npush, uint64_t &cacc) {
    constexpr uint32_t max_queue = BLOCK / G;
    uint32_t sel_done = 0;
    for (uint32_t run = 0; run < ST_SOLO_MAX_RUN; run++) {
        const uint32_t nq = ld_acq(&p.rec[n % REC_RING].nq);
        if (nq == 0 || nq > max_queue) break;
        st_select<G, QM>(p, n, 0, 1, cacc);
        st_solo_sync();
        const uint32_t mode = st_decide<QM>(p, n, prev);
        const uint64_t sel = ld_acq(&p.rec[n % REC_RING].sel);
        if (mode != 0 || (sel & 0xffffffffull) * G > ST_SOLO_MAX_UNITS) {
            sel_done = 1;
            break;
        }
        if (threadIdx.x == 0) st_record(p, n, 0);
        expand_items<G, QM, false>(p, n, L, sel, ~0u, 0, 1);
        st_solo_sync();
        npush++;
        prev = 0;
        n++;
    }
    if (threadIdx.x == 0) {
        p.bar->solo_n = n;
        p.bar->solo_sel = sel_done;
    }
}

// Writes the work counters this workgroup kept (threads 3..8, see st_select).
__device__ __forceinline__ void st_flush_counters(const StackParams &p, uint64_t cacc) {
    if (threadIdx.x >= 3 && threadIdx.x < 3 + ST_NCNT && cacc)
        atomicAdd(reinterpret_cast<unsigned long long *>(&p.cnt[threadIdx.x - 3]), static_cast<unsigned long long>(cacc));
}

template <int G, int QM>
__global__ __launch_bounds__(BLOCK) void k_stacked(StackParams p) {
    __shared__ StLds L;
    st_qv_setup(p.qv);
    GridBarrier *bar = p.bar;
    BarCtx bc;
    if (!barrier_register(bar, bc)) return;
    // a launch that continues after the phase kernels (every workgroup reads
    // the same words: the host wrote them before the launch)
    const bool resume = p.hand && ldc(&p.hand[HAND_RESUME]) != 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0 && !resume) {
        rec_clear(p.rec[0]);
        for (int i = 0; i < 4; i++) p.status[i] = 0;
        for (int i = 0; i < ST_NCNT; i++) p.cnt[i] = 0;
    }
    if (!grid_barrier(bar, bc)) return;
    // start pairs M_0 = Q_S x {source}: every source's bit in its start rows,
    // as candidates that level 0's select adds to P
    const QHeader &h = *s_qv.h;
    const uint32_t V = static_cast<uint32_t>(p.V);
    for (uint32_t i = resume ? ~0u : gthread(); i < static_cast<uint32_t>(p.B); i += gthreads()) {
        const uint32_t s = static_cast<uint32_t>(p.sources[i]);
        if (s >= V) {
            sviol(p);
            continue;
        }
        if (!h.smask) continue;
        const uint64_t bit = 1ull << (i & 63);
        uint32_t sm = h.smask;
        while (sm) {
            const uint32_t q = __ffs(sm) - 1;
            sm &= sm - 1;
            atomicOr(reinterpret_cast<unsigned long long *>(p.M[0] + rowi<G>(p, s, q) + (i >> 6)),
                     static_cast<unsigned long long>(bit));
        }
        if (sup_or<QM>(p.sup[0], s, h.smask) == 0) {
            const uint32_t pos = atomicAdd(&p.rec[0].nq, 1u);
            if (pos < V) p.q[0][pos] = static_cast<int32_t>(s);
            else sviol(p);
        }
    }
    if (!grid_barrier(bar, bc)) return;
    uint32_t n = 0, npush = 0, npull = 0, prev = 0, solo_at = ~0u;
    uint64_t last_pairs = 0, cacc = 0;
    bool resumed = false;  // level n's select was made by the phase kernels
    if (resume) {
        n = ldc(&p.hand[HAND_LEVEL]);
        npush = ldc(&p.hand[HAND_NPUSH]);
        npull = ldc(&p.hand[HAND_NPULL]);
        last_pairs = static_cast<uint64_t>(ldc(&p.hand[HAND_LAST_LO])) |
                     (static_cast<uint64_t>(ldc(&p.hand[HAND_LAST_HI])) << 32);
        resumed = true;
    }
    while (true) {
        const uint32_t nq = ld_acq(&p.rec[n % REC_RING].nq);
        if (nq == 0) break;
        bool selected = resumed;
        resumed = false;
        if (!selected && nq <= BLOCK / G && n != solo_at) {
            // a run of small levels in workgroup 0; the rest wait here
            solo_at = n;
            if (blockIdx.x == 0) st_solo_levels<G, QM>(p, n, L, prev, npush, cacc);
            if (!grid_barrier(bar, bc)) return;
            const uint32_t n2 = ld_acq(&bar->solo_n);
            if (n2 != n) {
                prev = 0;  // small levels are pushed
                last_pairs = ld_acq(&p.rec[(n2 - 1) % REC_RING].pairs);
            }
            n = n2;
            selected = ld_acq(&bar->solo_sel) != 0;
            if (!selected) continue;
        }
        if (!selected) {
            st_select<G, QM>(p, n, blockIdx.x, gridDim.x, cacc);
            if (!grid_barrier(bar, bc)) return;
        }
        LevelRec &R = p.rec[n % REC_RING];
        last_pairs = ld_acq(&R.pairs);
        const uint32_t mode = st_decide<QM>(p, n, prev);
        if (blockIdx.x == 0 && threadIdx.x == 0) st_record(p, n, mode);
        if (mode == 0 && p.handoff_edges && (ld_acq(&R.sel) & 0xffffffffull) >= p.handoff_edges &&
            (ld_acq(&R.sel) & 0xffffffffull) >= V / ST_SWEEP_DIV) {
            // a large push level: the phase kernels take over from here (the
            // same decision in every workgroup: all read R after the barrier)
            st_flush_counters(p, cacc);
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                p.hand[HAND_EXIT] = 1;
                p.hand[HAND_LEVEL] = n;
                p.hand[HAND_NPUSH] = npush;
                p.hand[HAND_NPULL] = npull;
            }
            return;
        }
        if (mode == 0) {
            const uint64_t sel = ld_acq(&R.sel);
            if ((sel & 0xffffffffull) >= V / ST_SWEEP_DIV) {
                // a large level: mark the candidates' state sets, then queue
                // them in vertex order
                expand_items<G, QM, false, true>(p, n, L, sel, ~0u, blockIdx.x, gridDim.x);
                if (!grid_barrier(bar, bc)) return;
                st_compact(p, n);
            } else {
                expand_items<G, QM, false>(p, n, L, sel, ~0u, blockIdx.x, gridDim.x);
            }
            if (!grid_barrier(bar, bc)) return;
            npush++;
        } else {
            if constexpr (QM <= 8) {
                // states the level can produce: successors of the frontier's states
                uint32_t su = ld_acq(&R.su), ns = 0;
                while (su) {
                    ns |= h.succ_any[__ffs(su) - 1];
                    su &= su - 1;
                }
                ns &= h.inmask;
                st_pull_rows<G>(p, n, ns);
                if (!grid_barrier(bar, bc)) return;
                const uint64_t hsel = ld_acq(&R.hsel);
                if (hsel) {
                    expand_items<G, 8, true>(p, n, L, hsel, ns, blockIdx.x, gridDim.x);
                    if (!grid_barrier(bar, bc)) return;
                }
            }
            npull++;
        }
        prev = mode;
        n++;
    }
    // this workgroup's share of the work counters (threads 3..8)
    st_flush_counters(p, cacc);
    // the last level may have found only visited pairs
    const uint32_t levels = (n > 0 && last_pairs == 0) ? n - 1 : n;
    st_final<G, QM>(p, n, levels);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.status[0] = levels;
        p.status[1] = npush;
        p.status[2] = npull;
        if (p.hand) p.hand[HAND_EXIT] = 0;
    }
}

// ------------------------------------------------------------ phase kernels
// Large push levels outside the persistent launch: each phase is a kernel of
// its own, so each gets the registers it needs alone (the expansion fits 128
// VGPRs, two 512-thread workgroups per CU, where the persistent kernel, which
// holds every phase, takes one), and kernel boundaries order the phases.
template <int G, int QM>
__global__ __launch_bounds__(st_expand_threads<G>()) __attribute__((amdgpu_waves_per_eu(st_expand_waves<G>())))
void k_st_expand(StackParams p, uint32_t n, uint32_t record) {
    __shared__ StLdsN<TILE / G + 1> L;
    st_qv_setup(p.qv);
    if (record && blockIdx.x == 0 && threadIdx.x == 0) st_record(p, n, 0);
    expand_items<G, QM, false, true, st_expand_upt<G>(), st_expand_threads<G>()>(p, n, L, ld_acq(&p.rec[n % REC_RING].sel), ~0u, blockIdx.x,
                                                   gridDim.x);
}

__global__ __launch_bounds__(BLOCK) void k_st_compact(StackParams p, uint32_t n) { st_compact(p, n); }

template <int G, int QM, bool COUNT>
__global__ __launch_bounds__(BLOCK) void k_st_select(StackParams p, uint32_t n) {
    st_qv_setup(p.qv);
    uint64_t cacc = 0;
    st_select<G, QM, COUNT>(p, n, blockIdx.x, gridDim.x, cacc);
    if constexpr (COUNT) st_flush_counters(p, cacc);
}

// The grid is sized to be resident on an otherwise idle GPU, and every
// persistent grid of the process takes its workgroups from a per-device
// budget of co-resident workgroups before it is launched, so an ordinary
// launch suffices; hipLaunchCooperativeKernel (which also guarantees
// residency against other processes) is the option.
template <int G, int QM>
static hipError_t launch_g(const StackParams &p, int grid, bool cooperative, hipStream_t s) {
    StackParams a = p;
    if (cooperative) {
        void *args[] = {&a};
        return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_stacked<G, QM>), dim3(grid), dim3(BLOCK),
                                          args, 0, s);
    }
    hipLaunchKernelGGL((k_stacked<G, QM>), dim3(grid), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

#define RPQ_STACKED_DISPATCH(G, QM, CALL8, CALL32)             \
    if ((QM) <= 8) {                                           \
        switch (G) {                                           \
            case 1: { constexpr int GG = 1; CALL8; } break;    \
            case 2: { constexpr int GG = 2; CALL8; } break;    \
            case 4: { constexpr int GG = 4; CALL8; } break;    \
            case 8: { constexpr int GG = 8; CALL8; } break;    \
            default: { constexpr int GG = 16; CALL8; } break;  \
        }                                                      \
    } else {                                                   \
        switch (G) {                                           \
            case 1: { constexpr int GG = 1; CALL32; } break;   \
            case 2: { constexpr int GG = 2; CALL32; } break;   \
            case 4: { constexpr int GG = 4; CALL32; } break;   \
            case 8: { constexpr int GG = 8; CALL32; } break;   \
            default: { constexpr int GG = 16; CALL32; } break; \
        }                                                      \
    }

hipError_t launch_stacked(int G, int QM, const StackParams &p, int grid, bool cooperative, hipStream_t s) {
    hipError_t e = hipSuccess;
    RPQ_STACKED_DISPATCH(G, QM, (e = launch_g<GG, 8>(p, grid, cooperative, s)),
                         (e = launch_g<GG, 32>(p, grid, cooperative, s)));
    return e;
}

// Workgroups for a phase kernel: as many as fit the GPU at once.
static int phase_grid(const void *kernel, int threads = BLOCK) {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per < 1) per = 1;
    return ncu * per;
}

template <int G, int QM>
static hipError_t st_expand_g(const StackParams &p, uint32_t n, bool record, hipStream_t s) {
    constexpr int NT = st_expand_threads<G>();
    static const int grid = phase_grid(reinterpret_cast<const void *>(&k_st_expand<G, QM>), NT);
    hipLaunchKernelGGL((k_st_expand<G, QM>), dim3(grid), dim3(NT), 0, s, p, n, record ? 1u : 0u);
    return hipGetLastError();
}

template <int G, int QM, bool COUNT>
static hipError_t st_select_g(const StackParams &p, uint32_t n, hipStream_t s) {
    static const int grid = phase_grid(reinterpret_cast<const void *>(&k_st_select<G, QM, COUNT>));
    hipLaunchKernelGGL((k_st_select<G, QM, COUNT>), dim3(grid), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_st_expand(int G, int QM, const StackParams &p, uint32_t n, bool record, hipStream_t s) {
    hipError_t e = hipSuccess;
    RPQ_STACKED_DISPATCH(G, QM, (e = st_expand_g<GG, 8>(p, n, record, s)), (e = st_expand_g<GG, 32>(p, n, record, s)));
    return e;
}

hipError_t launch_st_select(int G, int QM, const StackParams &p, uint32_t n, bool counters, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (counters)
        RPQ_STACKED_DISPATCH(G, QM, (e = st_select_g<GG, 8, true>(p, n, s)), (e = st_select_g<GG, 32, true>(p, n, s)))
    else
        RPQ_STACKED_DISPATCH(G, QM, (e = st_select_g<GG, 8, false>(p, n, s)), (e = st_select_g<GG, 32, false>(p, n, s)))
    return e;
}

hipError_t launch_st_compact(const StackParams &p, uint32_t n, hipStream_t s) {
    static const int grid = phase_grid(reinterpret_cast<const void *>(&k_st_compact));
    hipLaunchKernelGGL(k_st_compact, dim3(grid), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}

// The fixed device array behind rpq_multi_source_noalloc, in the module of
// the kernels that use it (so no module of its own is registered). Host code
// never passes `scratch` itself to a kernel: in host code the name is a
// host-side stand-in, and the device address comes from hipGetSymbolAddress
// below, once per device with that device current (each GPU holds its own
// copy at its own address from then until the process ends).
static __device__ __align__(256) uint8_t scratch[RPQ_NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch_address(void **ptr) { return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch)); }

int stacked_blocks_per_cu(int G, int QM) {
    int per = 0;
    hipError_t e = hipSuccess;
    RPQ_STACKED_DISPATCH(G, QM, (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_stacked<GG, 8>, BLOCK, 0)),
                         (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_stacked<GG, 32>, BLOCK, 0)));
    return e == hipSuccess ? per : -1;
}

int stacked_grid(int G, int QM) {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const int per = stacked_blocks_per_cu(G, QM);
    if (per < 1) return 0;
    return ncu * (per < PERSISTENT_BLOCKS_PER_CU ? per : PERSISTENT_BLOCKS_PER_CU);
}

}  // namespace rpq
