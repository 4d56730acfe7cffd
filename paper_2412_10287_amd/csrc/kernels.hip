// HIP kernels for one single-source query on gfx950 (64-lane wavefronts).
//
// One level of Alg. 1 (Sec. 4) computes
//     M' = ( sum_a (N^a)^T M G^a ) masked by not-P,      P = P + M'
// over the Boolean semiring. The kernels never form a matrix. Per vertex the
// |Q| states of M and P are one bit-packed word (1, 2 or 4 bytes), and a level
// runs as two phases separated by a grid barrier:
//
//  select  every candidate vertex w (one that received state bits in the
//          previous expansion) is masked by P: its new states M[w] & ~P[w]
//          are added to P and become w's frontier word. Then, for each used
//          symbol u, the product (N^u)^T M restricted to column w is the
//          successor set succ_u(M[w]) (a few table ORs); each non-empty one
//          with a u-row at w becomes a push item (neighbour range, state set).
//          This applies the small NFA factor first, the evaluation order
//          Sec. 4 recommends.
//  push    the items' edges are spread evenly over the grid; each edge (v, w)
//          drops the item's states already in P[w] (a load) and ORs the rest
//          into the next level's word of w with one atomic; the first writer
//          of that word appends w to the next candidate queue (wave ballot +
//          popc, one reservation per workgroup and step of four edges per
//          lane).
//  pull    used instead of push on dense levels: every vertex w with states
//          still unvisited scans its reverse neighbours under the symbols that
//          can reach those states and stops as soon as all are found.
//
// Masking by P in the next select instead of with an atomic on P during the
// scatter takes one atomic round trip off every edge; random 32-bit atomics
// are the most expensive operation of the traversal on MI355X.
//
// Inverse symbols a^- read the transposed adjacency (Sec. 3: G^{a^-} = (G^a)^T):
// the graph store holds both directions, and the label -> symbol tables map an
// IN segment to the inverse symbol of its label.
//
// The whole traversal runs as one persistent launch with grid barriers
// between phases (no host round trip per level); the same phase code is also
// launched kernel by kernel for the host-driven loop. Inside the persistent
// launch, runs of small levels execute in workgroup 0 alone (solo_levels),
// and a mid-size level after a push level is fused: each workgroup pushes
// the edges of its own items right after selecting them, one grid barrier
// per level (block_reserve_fused).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "rpq_internal.h"

namespace rpq {

// The running query's tables, for every phase of this file's kernels: a copy
// in LDS when the block fits (the persistent kernel), else the global block.
__shared__ QueryView s_qv;
__shared__ __align__(16) uint8_t s_qc[QC_LDS_BYTES];

// Sets s_qv (copying the block into s_qc when TO_LDS and it fits). Every
// thread of the workgroup calls it; it ends with a workgroup barrier.
template <bool TO_LDS>
__device__ __forceinline__ void qv_setup(const QueryView &qv) {
    bool fits = false;
    uint32_t nsym = 0;
    if constexpr (TO_LDS) {
        nsym = qv.h->nsym;
        const size_t qb = qconst_bytes(nsym);
        fits = qb <= QC_LDS_BYTES;
        if (fits) {
            const uint4 *src = reinterpret_cast<const uint4 *>(qv.h);
            uint4 *dst = reinterpret_cast<uint4 *>(s_qc);
            for (uint32_t i = threadIdx.x; i < (qb + 15) / 16; i += blockDim.x) dst[i] = src[i];
        }
    }
    if (threadIdx.x == 0) {
        if constexpr (TO_LDS) s_qv = fits ? qconst_view(s_qc, nsym) : qv;
        else s_qv = qv;
    }
    __syncthreads();
}

// Records a violated invariant (an index read from device memory out of
// range); the access is skipped and the host reports the query as failed.
// Host-visible status word k (pinned host memory; see StateView::hstat).
__device__ __forceinline__ void hstat_store(const Params &p, int k, uint32_t v) {
    if (p.st.hstat) __hip_atomic_store(p.st.hstat + k, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void flag_violation(const Params &p) {
    atomicAdd(&p.st.status[3], 1u);
    hstat_store(p, 3, 1u);
}

// Runs of small levels (solo_levels) execute in workgroup 0 alone; their
// queues, reservation cursors and level totals live in LDS (SoloLds) rather
// than in the level records, so such a level makes no global atomic and
// reads nothing global but state words and the graph.
constexpr uint32_t SOLO_MAX_QUEUE = 512;  // candidate queue entries of a small level
constexpr uint32_t SOLO_MAX_EDGES = 1024;  // push edges of a small level (more take one CU longer than the grid)
constexpr uint32_t SOLO_MAX_RUN = 2048;    // levels per run (the waiting workgroups' barrier times out after 5 s)

struct SoloLds {
    uint64_t sel, pairs;           // the level's reservations ((items << 32) | edges) and pairs
    uint32_t nfront, su, prev_mode;
    int32_t q[2][SOLO_MAX_QUEUE];  // candidate queues of levels n and n + 1, by parity
};

// ---------------------------------------------------------------- phases
// Run by every thread of workgroup 0 (the caller orders its stores before
// level 0 reads them).
template <int W>
__device__ __forceinline__ void init_phase(const Params &p) {
    if (blockIdx.x != 0) return;
    const QHeader &h = *s_qv.h;
    LevelRec *r = p.st.rec;
    const uint32_t sm = h.smask;
    if (threadIdx.x == 0) {
        // records are cleared two levels ahead (select_phase): levels 0 and 1 here
        rec_clear(r[0]);
        rec_clear(r[1]);
        for (int i = 0; i < 4; i++) p.st.cnt[i] = 0;
        for (int i = 0; i < 4; i++) p.st.status[i] = 0;
    }
    if (!sm) return;
    // M_0 = Q_S x V_s (V_s = {source}, or the distinct vertices of a source
    // set), as candidates that level 0's select adds to P
    if (p.nsrc == 0) {
        if (threadIdx.x == 0) {
            st_state<W>(p.st.M[0], p.source, sm);
            p.st.q[0][0] = p.source;
            r[0].nq = 1;
        }
        return;
    }
    const uint32_t V = static_cast<uint32_t>(p.g.V);
    for (uint32_t i = threadIdx.x; i < p.nsrc; i += blockDim.x) {
        const uint32_t v = static_cast<uint32_t>(p.srcset[i]);
        if (v < V) {
            st_state<W>(p.st.M[0], v, sm);
            p.st.q[0][i] = static_cast<int32_t>(v);
        } else {
            flag_violation(p);
            p.st.q[0][i] = 0;
        }
    }
    if (threadIdx.x == 0) r[0].nq = p.nsrc;
}

// Zeroes the state words that level k's queue entries point to in M[k & 1]
// (its candidate and frontier words), eight entries per thread and step with
// all loads before the stores (one workgroup alone may clear a long queue).
template <int W, bool LQ = false>
__device__ __forceinline__ void clear_level_words(const Params &p, uint32_t k, uint32_t nk, uint32_t bid,
                                                  uint32_t nblk, const int32_t *lq = nullptr) {
    const uint32_t V = static_cast<uint32_t>(p.g.V);
    if (nk > V) nk = V;
    uint32_t *M = p.st.M[k & 1];
    const int32_t *q = p.st.q[k & 1];
    const uint32_t stride = nblk * BLOCK;
    for (uint32_t i0 = bid * BLOCK + threadIdx.x; i0 < nk; i0 += 8 * stride) {
        uint32_t vv[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const uint32_t i = i0 + j * stride;
            // LQ: the queue's copy in LDS (a solo level's)
            vv[j] = i < nk ? static_cast<uint32_t>(LQ ? lq[i] : ldc(&q[i])) : 0u;
        }
#pragma unroll
        for (int j = 0; j < 8; j++) {
            if (i0 + j * stride >= nk) continue;
            if (vv[j] < V) st_state<W>(M, vv[j], 0);
            else flag_violation(p);
        }
    }
}

template <int W, bool SOLO = false>
__device__ __forceinline__ uint32_t push_range(const Params &p, uint32_t n, const uint32_t *s_eb,
                                               const uint32_t *s_beg, const uint32_t *s_mask, uint32_t cnt,
                                               uint32_t ubase, uint32_t uend, int32_t *lq = nullptr);

// A mid-size level after a push level is fused: each workgroup pushes the
// edges of its own items right after selecting them (from LDS, up to
// FUSE_LOCAL_EDGES edges and TILE + 1 items), and only the items beyond that
// budget are reserved globally and pushed over the grid after the barrier.
// One grid barrier less per such level; the level is always pushed.
constexpr uint32_t FUSE_LOCAL_EDGES = 2 * TILE;
constexpr uint32_t FUSE_V_DIV = 32;  // fused while the queue holds at most V / 32 candidates

// The reservation of one select round of a fused level: the round goes to
// the workgroup's own items (cursor `local`, in registers) while they fit
// the budget, else to the level's global items (counter `glob`). Packed
// (items << 32) | edges as in block_reserve; `is_local` tells which.
__device__ __forceinline__ bool block_reserve_fused(uint64_t wtot, bool more, uint64_t &local, uint64_t *glob,
                                                    uint64_t &base, bool &is_local) {
    __shared__ uint64_t s_w[NWAVE];
    __shared__ uint32_t s_more[NWAVE];
    __shared__ uint64_t s_base;
    const uint32_t wave = threadIdx.x >> 6;
    const bool wmore = __ballot(more) != 0;
    if (lane_id() == 0) {
        s_w[wave] = wtot;
        s_more[wave] = wmore ? 1u : 0u;
    }
    __syncthreads();
    uint64_t off = 0, tot = 0;
    uint32_t any = 0;
#pragma unroll
    for (int k = 0; k < NWAVE; k++) {
        const uint64_t x = s_w[k];
        if (static_cast<uint32_t>(k) < wave) off += x;
        tot += x;
        any |= s_more[k];
    }
    const uint64_t after = local + tot;
    is_local = (after >> 32) <= static_cast<uint64_t>(TILE) + 1 && static_cast<uint32_t>(after) <= FUSE_LOCAL_EDGES &&
               static_cast<uint32_t>(after) >= static_cast<uint32_t>(local);
    if (!is_local && threadIdx.x == 0 && tot) s_base = atomic_add_any(glob, tot);
    __syncthreads();  // s_w read everywhere, s_base published
    if (is_local) {
        base = local + off;
        local = after;
    } else {
        base = tot ? s_base + off : 0ull;
    }
    return any != 0;
}

// Candidates -> frontier -> push items. Each candidate w gets its new states
// S = M[w] & ~P[w] (added to P); for each used symbol u, succ_u(S) is the
// column w of (N^u)^T M, and when it is non-empty and w has u-neighbours,
// (w, u) becomes an item carrying the neighbour range and succ_u(S). Items are
// reserved per workgroup with one 64-bit atomic that counts items (high half)
// and edges (low half) together, so item order and edge numbering agree.
//
// nq is the level's queue length (its record's nq).
//
// SOLO: workgroup 0 alone runs the level (bid 0, nblk 1). When solo_lq the
// queue comes from so->q; reservations advance a cursor in registers; the
// items are also kept in s_eb, s_beg and s_mask (the first TILE + 1 of them),
// and the level's totals go to `so` as well as, with plain stores, to its
// level record.
//
// FUSED (grid, a mid-size level that is pushed): rounds that fit the
// workgroup's budget keep their items in s_eb, s_beg and s_mask (local
// numbering) and are pushed at the end by this workgroup; the frontier words
// are cleared at once (a pushed level never reads them again); the local
// items and edges are added to the record's hsel for the statistics.
template <int W, bool SOLO = false, bool FUSED = false>
__device__ __forceinline__ void select_phase(const Params &p, uint32_t n, uint32_t nq, uint32_t bid, uint32_t nblk,
                                             SoloLds *so = nullptr, bool solo_lq = false, uint32_t *s_eb = nullptr,
                                             uint32_t *s_beg = nullptr, uint32_t *s_mask = nullptr) {
    static_assert(!(SOLO && FUSED), "one mode");
    const GraphView &g = p.g;
    const QueryView &qv = s_qv;
    const QHeader &h = *qv.h;
    LevelRec *rec = p.st.rec;
    LevelRec &R = rec[n % REC_RING];
    const uint32_t V = static_cast<uint32_t>(g.V);
    if (nq > V) {
        if (bid == 0 && threadIdx.x == 0) flag_violation(p);
        nq = V;
    }
    if (bid == 0 && threadIdx.x == 0) {
        // the record of level n+2: level n+1's is already clear (a fused level's
        // pushes append to it while other workgroups still select)
        rec_clear(rec[(n + 2) % REC_RING]);
        if (n < LVL_COUNT_CAP) p.st.lvl[static_cast<uint64_t>(n) * LVL_STRIDE + 3] = wall_clock64();
    }
    // frontier words of level n-1 live in the buffer level n writes: after a
    // pull level they are cleared here (after a push level, that level's
    // push phase has cleared them already). A solo level after another one
    // follows a push level.
    const uint32_t prev_mode = (n >= 1 && !(SOLO && solo_lq)) ? ld_acq(&rec[(n - 1) % REC_RING].mode) : 0u;
    if (prev_mode != 0) clear_level_words<W>(p, n - 1, ld_acq(&rec[(n - 1) % REC_RING].nq), bid, nblk);
    const int32_t *qc = p.st.q[n & 1];
    uint64_t run_sel = 0;  // SOLO: the reservation cursor; FUSED: the workgroup's own items
    uint32_t *Mc = p.st.M[n & 1];
    uint32_t *P = p.st.P;
    const uint32_t nsym = h.nsym;
    uint64_t c_pe = 0, c_sc = 0, c_sd = 0, pairs = 0;
    uint32_t nfront = 0, su = 0;
    // With at most SYM_BATCH used symbols, all of them are looked up in one
    // round, and their rank words are loaded together with the state words
    // (before S is known): one dependent round trip less per level.
    const bool few_sym = nsym <= static_cast<uint32_t>(SYM_BATCH);
    // Candidates [q0, q1) of this workgroup, BLOCK per round, every
    // nblk * BLOCK (the grid and one workgroup). A fused level spreads its
    // candidates over the whole grid in wave-sized chunks instead, so each
    // workgroup's own push stays short.
    uint32_t q0 = bid * BLOCK, q1 = nq, qstep = nblk * BLOCK;
    if constexpr (FUSED) {
        uint32_t chunk = (nq + nblk - 1) / nblk;
        chunk = (chunk + 63) & ~63u;
        q0 = bid * chunk < nq ? bid * chunk : nq;
        q1 = q0 + chunk < nq ? q0 + chunk : nq;
        qstep = BLOCK;
    }
    // workgroup-uniform loop: item reservations are made per workgroup
    for (uint32_t bbase = q0; bbase < q1; bbase += qstep) {
        const uint32_t i = bbase + threadIdx.x;
        uint32_t v = 0, S = 0;
        RankWordD rwp[SYM_BATCH];
        if (i < q1) {
            v = static_cast<uint32_t>(SOLO && solo_lq ? so->q[n & 1][i] : ldc(&qc[i]));
            if (v < V) {
                if (few_sym) {
#pragma unroll
                    for (int j = 0; j < SYM_BATCH; j++)
                        if (static_cast<uint32_t>(j) < nsym) rwp[j] = g.rankw[qv.push_w[j] + (v >> 6)];
                }
                // the complement mask of Alg. 1, then P = P + M
                const uint32_t c = ld_state<W>(Mc, v);
                const uint32_t pv = ld_state<W>(P, v);
                S = c & ~pv;
                if (S) st_state<W>(P, v, pv | S);
                // shortest accepted walk: the first level at which v holds a
                // final state (levels only grow, so the first is the least)
                if (p.dist && (S & h.fmask) && !(pv & h.fmask)) p.dist[v] = static_cast<int32_t>(n);
                if constexpr (FUSED) {
                    if (c) st_state<W>(Mc, v, 0u);
                } else if (S != c) {
                    st_state<W>(Mc, v, S);
                }
                pairs += __popc(S);
                nfront += S != 0;
                su |= S;
            } else {
                flag_violation(p);
                v = 0;
            }
        }
        // only the symbols with a transition out of S can give an item; the
        // rounds continue while any lane of the workgroup has symbols left
        SymSet Rs;
        if (!few_sym) Rs = symbols_of(qv, S, nsym);
        while (true) {
            uint32_t us[SYM_BATCH], sp[SYM_BATCH], beg[SYM_BATCH], len[SYM_BATCH];
            RankWordD rw[SYM_BATCH];
            bool more = false;
            if (few_sym) {
#pragma unroll
                for (int j = 0; j < SYM_BATCH; j++) {
                    us[j] = static_cast<uint32_t>(j) < nsym ? static_cast<uint32_t>(j) : nsym;
                    sp[j] = us[j] < nsym ? succ_of(qv.succ, us[j], S) : 0u;
                    if (sp[j]) rw[j] = rwp[j];
                }
            } else {
#pragma unroll
                for (int j = 0; j < SYM_BATCH; j++) us[j] = symbol_pop(Rs);
#pragma unroll
                for (int k = 0; k < SYM_WORDS; k++) more = more || Rs.w[k] != 0;
#pragma unroll
                for (int j = 0; j < SYM_BATCH; j++) {
                    sp[j] = us[j] < nsym ? succ_of(qv.succ, us[j], S) : 0u;
                    if (sp[j]) rw[j] = g.rankw[qv.push_w[us[j]] + (v >> 6)];
                }
            }
            uint32_t cnt = 0, tot = 0, nscan = 0;
#pragma unroll
            for (int j = 0; j < SYM_BATCH; j++) {
                len[j] = 0;
                uint32_t e;
                nscan += sp[j] != 0;
                if (sp[j] && row_range(g, rw[j], qv.push_r[us[j]], v, beg[j], e)) {
                    if (e > beg[j] && e <= g.ncol) len[j] = e - beg[j];
                    else if (e != beg[j]) flag_violation(p);
                }
                if (len[j]) {
                    cnt++;
                    tot += len[j];
                    if (h.counters) c_pe += static_cast<uint64_t>(count_succ(qv.succ, us[j], S)) * len[j];
                }
            }
            if (h.counters) {
                // a scan is charged its row-pointer lookup whether or not the
                // row exists
                c_sc += nscan;
                c_sd += tot;
            }
            uint64_t wtot;
            const uint64_t ex = wave_excl_scan((static_cast<uint64_t>(cnt) << 32) | tot, wtot);
            uint64_t wbase;
            bool bmore, to_lds = SOLO;
            if constexpr (SOLO) bmore = block_reserve_local<uint64_t>(wtot, more, run_sel, wbase);
            else if constexpr (FUSED) bmore = block_reserve_fused(wtot, more, run_sel, &R.sel, wbase, to_lds);
            else bmore = block_reserve<uint64_t>(wtot, more, &R.sel, wbase);
            if (FUSED && to_lds && cnt) {
                // this workgroup's own items (local numbering, within the budget)
                const uint64_t mine = wbase + ex;
                uint32_t idx = static_cast<uint32_t>(mine >> 32);
                uint32_t eb = static_cast<uint32_t>(mine);
#pragma unroll
                for (int j = 0; j < SYM_BATCH; j++) {
                    if (!len[j]) continue;
                    if (idx <= static_cast<uint32_t>(TILE)) {
                        s_eb[idx] = eb;
                        s_beg[idx] = beg[j];
                        s_mask[idx] = sp[j];
                    } else {
                        flag_violation(p);
                    }
                    idx++;
                    eb += len[j];
                }
            } else if (cnt) {
                const uint64_t mine = wbase + ex;
                uint32_t idx = static_cast<uint32_t>(mine >> 32);
                uint32_t eb = static_cast<uint32_t>(mine);
#pragma unroll
                for (int j = 0; j < SYM_BATCH; j++) {
                    if (!len[j]) continue;
                    if (idx < p.st.item_cap) {
                        p.st.it_ebase[idx] = eb;
                        p.st.it_beg[idx] = beg[j];
                        p.st.it_mask[idx] = sp[j];
                    } else {
                        flag_violation(p);
                    }
                    if (SOLO && idx <= static_cast<uint32_t>(TILE)) {
                        s_eb[idx] = eb;
                        s_beg[idx] = beg[j];
                        s_mask[idx] = sp[j];
                    }
                    // this item owns the tiles whose first edge falls inside it
                    const uint32_t k1 = (eb + len[j] - 1) / TILE;
                    for (uint32_t k = (eb + TILE - 1) / TILE; k <= k1; k++) {
                        if (k < p.st.tile_cap) p.st.tile_first[k] = idx;
                        else { flag_violation(p); break; }
                    }
                    idx++;
                    eb += len[j];
                }
            }
            if (!bmore) break;
        }
    }
    // level totals: one atomic per workgroup and field
    const uint64_t nf = wave_sum(static_cast<uint64_t>(nfront));
    {
        const uint64_t v[3] = {wave_sum(pairs), nf, wave_or(su)};
        const uint64_t t = block_reduce<3>(v, 4u);
        if constexpr (SOLO) {
            // the only workgroup: plain stores, into the record for the grid
            // (should it take the level over) and into LDS for workgroup 0
            if (threadIdx.x == 0) {
                so->pairs = t;
                so->sel = run_sel;
                so->prev_mode = prev_mode;
                R.pairs = t;
                R.sel = run_sel;
            }
            if (threadIdx.x == 1) {
                so->nfront = static_cast<uint32_t>(t);
                R.nfront = static_cast<uint32_t>(t);
            }
            if (threadIdx.x == 2) {
                so->su = static_cast<uint32_t>(t);
                R.su = static_cast<uint32_t>(t);
            }
        } else if (t) {
            if (threadIdx.x == 0) atomicAdd(reinterpret_cast<unsigned long long *>(&R.pairs), (unsigned long long)t);
            if (threadIdx.x == 1) atomicAdd(&R.nfront, static_cast<uint32_t>(t));
            if (threadIdx.x == 2) atomicOr(&R.su, static_cast<uint32_t>(t));
        }
    }
    if (h.counters) {
        const uint64_t v[4] = {wave_sum(c_pe), wave_sum(c_sc), wave_sum(c_sd), nf};
        const uint64_t t = block_reduce<4>(v, 0u);
        if (t && threadIdx.x < 4)
            atomicAdd(reinterpret_cast<unsigned long long *>(&p.st.cnt[threadIdx.x]), (unsigned long long)t);
    }
    if constexpr (FUSED) {
        // this workgroup's own items: their edges pushed now
        if (run_sel >> 32) {
            __syncthreads();  // the items are in LDS
            push_range<W>(p, n, s_eb, s_beg, s_mask, static_cast<uint32_t>(run_sel >> 32), 0u,
                          static_cast<uint32_t>(run_sel));
            if (threadIdx.x == 0) atomic_add_any(&R.hsel, run_sel);
            __syncthreads();  // the LDS items are free again
        }
    }
}

// Level n's totals once its select phase is complete, read by every thread
// at once (one round trip): its push reservations, pairs, frontier vertices,
// queue length and the direction of level n-1.
struct LevelInfo {
    uint64_t sel, pairs;
    uint32_t nfront, nq, prev_mode;
};

__device__ __forceinline__ LevelInfo level_info(const Params &p, uint32_t n) {
    const LevelRec &R = p.st.rec[n % REC_RING];
    LevelInfo li;
    li.sel = ld_acq(&R.sel);
    li.pairs = ld_acq(&R.pairs);
    li.nfront = ld_acq(&R.nfront);
    li.nq = ld_acq(&R.nq);
    li.prev_mode = n ? ld_acq(&p.st.rec[(n - 1) % REC_RING].mode) : 0u;
    return li;
}

// Level n's statistics (one thread).
__device__ __forceinline__ void record_level(const Params &p, uint32_t n, uint32_t mode, const LevelInfo &li) {
    p.st.rec[n % REC_RING].mode = mode;
    if (n < LVL_COUNT_CAP) {
        uint64_t *L = p.st.lvl + static_cast<uint64_t>(n) * LVL_STRIDE;
        L[0] = li.pairs;
        L[1] = li.nfront;
        L[2] = li.sel;
        L[4] = wall_clock64();
    }
}

// push (0) or pull (1) for level n; every workgroup computes the same answer
__device__ __forceinline__ uint32_t decide(const Params &p, const LevelInfo &li) {
    const QHeader &h = *s_qv.h;
    if (h.force == 1) return 0;
    if (h.force == 2) return 1;
    if (!(h.alpha > 0.f)) return 0;
    const uint64_t T = li.sel & 0xffffffffull;
    if (li.prev_mode == 0) return static_cast<double>(T) * h.alpha > static_cast<double>(h.e_rel) ? 1u : 0u;
    return static_cast<double>(li.nfront) * h.beta < static_cast<double>(p.g.V) ? 0u : 1u;
}

// Edges [ubase, uend) of the items staged in LDS (cnt of them), four per
// thread and step: all four loads of col, then of P, then the atomics, then
// one queue reservation per workgroup. Per edge (v, w) with successor set S' the
// states of S' not yet in P[w] (the complement mask) are ORed into the next
// level's word of w; the first writer appends w to the candidate queue.
// SOLO (workgroup 0 alone): the queue length is a cursor in registers, the
// entries also go to lq (the first SOLO_MAX_QUEUE), and the length is returned.
template <int W, bool SOLO>
__device__ __forceinline__ uint32_t push_range(const Params &p, uint32_t n, const uint32_t *s_eb,
                                               const uint32_t *s_beg, const uint32_t *s_mask, uint32_t cnt,
                                               uint32_t ubase, uint32_t uend, int32_t *lq) {
    const uint32_t V = static_cast<uint32_t>(p.g.V);
    const uint32_t *P = p.st.P;
    uint32_t *Mn = p.st.M[(n + 1) & 1];
    int32_t *qn = p.st.q[(n + 1) & 1];
    uint32_t *qlen = &p.st.rec[(n + 1) % REC_RING].nq;
    const uint32_t *col = p.g.col;
    const uint32_t tid = threadIdx.x;
    static_assert(TILE == 4 * BLOCK, "four edges per thread and step");
    uint32_t run_q = 0;
    // the halving steps of the item search depend on cnt alone (the same in
    // every lane): a uniform loop of ceil(log2(cnt)) steps, no step for one item
    const uint32_t ucnt = __builtin_amdgcn_readfirstlane(cnt);
    for (uint32_t ub = ubase; ub < uend; ub += TILE) {
        uint32_t w[4], sp[4], lo[4], tt[4];
        // item holding edge t: the last staged item with s_eb <= t (s_eb[0]
        // <= ubase); lanes past uend search for uend - 1 and drop the result
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint32_t t = ub + k * BLOCK + tid;
            tt[k] = t < uend ? t : uend - 1;
            lo[k] = 0;
        }
        for (uint32_t len = ucnt; len > 1;) {
            const uint32_t half = len >> 1;
#pragma unroll
            for (int k = 0; k < 4; k++)
                if (s_eb[lo[k] + half] <= tt[k]) lo[k] += half;
            len -= half;
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint32_t t = ub + k * BLOCK + tid;
            w[k] = V;
            sp[k] = 0;
            if (t < uend) {
                const uint32_t pos = s_beg[lo[k]] + (t - s_eb[lo[k]]);
                sp[k] = s_mask[lo[k]];
                if (pos < p.g.ncol) w[k] = col[pos];
                else flag_violation(p);
                if (w[k] >= V && pos < p.g.ncol) {
                    flag_violation(p);
                    w[k] = V;
                }
            }
        }
        uint32_t cand[4];
#pragma unroll
        for (int k = 0; k < 4; k++) cand[k] = w[k] < V ? sp[k] & ~ld_state<W>(P, w[k]) : 0u;
        bool first[4];
#pragma unroll
        for (int k = 0; k < 4; k++) first[k] = cand[k] ? or_state<W>(Mn, w[k], cand[k]) == 0 : false;
        bool ok;
        if constexpr (SOLO)
            ok = block_append4_local(first[0], static_cast<int32_t>(w[0]), first[1], static_cast<int32_t>(w[1]),
                                     first[2], static_cast<int32_t>(w[2]), first[3], static_cast<int32_t>(w[3]), lq,
                                     SOLO_MAX_QUEUE, qn, V, run_q);
        else
            ok = block_append4(first[0], static_cast<int32_t>(w[0]), first[1], static_cast<int32_t>(w[1]), first[2],
                               static_cast<int32_t>(w[2]), first[3], static_cast<int32_t>(w[3]), qn, qlen, V);
        if (!ok) flag_violation(p);
    }
    return run_q;
}

// Items -> edges, spread evenly over the grid. Few items: every workgroup
// stages all of them and takes an even, wave-aligned share of the edges, so
// small levels use the whole chip. Otherwise tile k holds edges
// [k*TILE, (k+1)*TILE) and its items are staged in LDS; with fewer tiles than
// workgroups each tile is split into parts of at least a wave's worth.
template <int W>
__device__ __forceinline__ void push_phase(const Params &p, uint32_t n, const LevelInfo &li, uint32_t *s_eb,
                                           uint32_t *s_beg, uint32_t *s_mask, uint32_t bid, uint32_t nblk,
                                           bool clear = true) {
    // the push direction never reads this level's words of M[n & 1] again
    // (items carry the successor sets): clear them now, with stores that
    // overlap the push; level n+1's expansion writes this buffer (a fused
    // level's select has cleared them already)
    if (clear) clear_level_words<W>(p, n, li.nq, bid, nblk);
    const uint64_t sel = li.sel;
    const uint32_t nitems = static_cast<uint32_t>(sel >> 32);
    const uint32_t T = static_cast<uint32_t>(sel);
    if (T == 0 || nitems == 0) return;
    if (nitems > p.st.item_cap) {
        if (bid == 0 && threadIdx.x == 0) flag_violation(p);
        return;
    }
    const uint32_t tid = threadIdx.x;
    if (nitems <= static_cast<uint32_t>(TILE)) {
        uint32_t per = (T + nblk - 1) / nblk;
        per = (per + 63) & ~63u;
        const uint64_t b0 = static_cast<uint64_t>(bid) * per;
        if (b0 >= T) return;  // no edges for this workgroup: nothing to stage
        const uint32_t b1 = b0 + per < T ? static_cast<uint32_t>(b0 + per) : T;
        for (uint32_t j = tid; j < nitems; j += BLOCK) {
            s_eb[j] = ldc(&p.st.it_ebase[j]);
            s_beg[j] = ldc(&p.st.it_beg[j]);
            s_mask[j] = ldc(&p.st.it_mask[j]);
        }
        __syncthreads();
        push_range<W>(p, n, s_eb, s_beg, s_mask, nitems, static_cast<uint32_t>(b0), b1);
        __syncthreads();
        return;
    }
    const uint32_t ntiles = (T + TILE - 1) / TILE;
    uint32_t sub = 1;
    while (sub < TILE / 64 && ntiles * sub * 2 <= nblk) sub *= 2;
    const uint32_t part = TILE / sub;
    for (uint32_t vt = bid; vt < ntiles * sub; vt += nblk) {
        const uint32_t tile = vt / sub, k = vt % sub;
        uint32_t i0 = tile < p.st.tile_cap ? ldc(&p.st.tile_first[tile]) : 0u;
        uint32_t i1 = (tile + 1 < ntiles && tile + 1 < p.st.tile_cap) ? ldc(&p.st.tile_first[tile + 1]) : nitems - 1;
        if (i0 >= nitems || i1 >= nitems || i1 < i0 || i1 - i0 > static_cast<uint32_t>(TILE)) {
            if (tid == 0) flag_violation(p);
            i0 = i1 = 0;
        }
        const uint32_t cnt = i1 - i0 + 1;  // <= TILE + 1
        for (uint32_t j = tid; j < cnt; j += BLOCK) {
            s_eb[j] = ldc(&p.st.it_ebase[i0 + j]);
            s_beg[j] = ldc(&p.st.it_beg[i0 + j]);
            s_mask[j] = ldc(&p.st.it_mask[i0 + j]);
        }
        __syncthreads();
        const uint32_t u0 = tile * TILE + k * part;
        const uint32_t u1 = u0 + part < T ? u0 + part : T;
        if (u0 < u1) push_range<W>(p, n, s_eb, s_beg, s_mask, cnt, u0, u1);
        __syncthreads();
    }
}

// Dense levels: every vertex w with states U that it lacks and the level can
// still produce looks, per used symbol u whose predecessor set pred_u(U) is
// non-empty, through its reverse u-neighbours v, ORs succ_u(M[v]) & U and stops
// once all of U is found. Each w is owned by one thread (light vertices) or
// one wavefront (vertices with more than PULL_LIGHT such neighbours, queued
// per workgroup in LDS and scanned 64 neighbours at a time): no atomics on P.
constexpr uint32_t PULL_LIGHT = 64;
constexpr uint32_t PULL_HEAVY_CAP = 512;

template <int W>
__device__ __forceinline__ uint32_t pull_rows(const Params &p, uint32_t w, uint32_t U, uint32_t u0,
                                              uint32_t *beg, uint32_t *end) {
    // row ranges of w for symbols u0 .. u0+SYM_BATCH-1 in the pull direction;
    // returns the summed length (0 for symbols that cannot reach U)
    const GraphView &g = p.g;
    const QueryView &qv = s_qv;
    const uint32_t nsym = qv.h->nsym;
    uint32_t pu[SYM_BATCH];
    RankWordD rw[SYM_BATCH];
#pragma unroll
    for (int j = 0; j < SYM_BATCH; j++) {
        const uint32_t u = u0 + j;
        pu[j] = u < nsym ? succ_of(qv.pred, u, U) : 0u;
        if (pu[j]) rw[j] = g.rankw[qv.pull_w[u] + (w >> 6)];
    }
    uint32_t tot = 0;
#pragma unroll
    for (int j = 0; j < SYM_BATCH; j++) {
        beg[j] = end[j] = 0;
        if (pu[j] && row_range(g, rw[j], qv.pull_r[u0 + j], w, beg[j], end[j])) {
            if (end[j] > g.ncol || end[j] < beg[j]) {
                flag_violation(p);
                beg[j] = end[j] = 0;
            }
        } else {
            beg[j] = end[j] = 0;
        }
        tot += end[j] - beg[j];
    }
    return tot;
}

template <int W>
__device__ __forceinline__ void pull_phase(const Params &p, uint32_t n, uint32_t *s_hw, uint32_t *s_hu, uint32_t *s_hp,
                           uint32_t *s_hn) {
    const GraphView &g = p.g;
    const QueryView &qv = s_qv;
    const QHeader &h = *qv.h;
    LevelRec *rec = p.st.rec;
    // states that can appear in the next frontier at all
    uint32_t su = ld_acq(&rec[n % REC_RING].su), ns = 0;
    while (su) {
        ns |= h.succ_any[__ffs(su) - 1];
        su &= su - 1;
    }
    ns &= h.inmask;
    const uint32_t *Mc = p.st.M[n & 1];
    uint32_t *Mn = p.st.M[(n + 1) & 1];
    int32_t *qn = p.st.q[(n + 1) & 1];
    const uint32_t *P = p.st.P;
    LevelRec &RN = rec[(n + 1) % REC_RING];
    const uint32_t lane = lane_id();
    const uint32_t V = static_cast<uint32_t>(g.V);
    const uint32_t nsym = h.nsym;
    if (threadIdx.x == 0) *s_hn = 0;
    __syncthreads();
    // workgroup-uniform loop: queue reservations are made per workgroup
    for (uint32_t bbase = blockIdx.x * BLOCK; bbase < V; bbase += gridDim.x * BLOCK) {
        const uint32_t w = bbase + threadIdx.x;
        uint32_t acc = 0;
        if (w < V) {
            const uint32_t pw = ld_state<W>(P, w);
            const uint32_t U = ns & ~pw;
            bool deferred = false;
            if (U) {
                // total work first: heavy vertices go to the workgroup's list
                uint32_t beg0[SYM_BATCH], end0[SYM_BATCH];
                uint32_t deg = pull_rows<W>(p, w, U, 0, beg0, end0);
                for (uint32_t u0 = SYM_BATCH; u0 < nsym && deg <= PULL_LIGHT; u0 += SYM_BATCH) {
                    uint32_t beg[SYM_BATCH], end[SYM_BATCH];
                    deg += pull_rows<W>(p, w, U, u0, beg, end);
                }
                if (deg > PULL_LIGHT) {
                    const uint32_t slot = atomicAdd(s_hn, 1u);
                    if (slot < PULL_HEAVY_CAP) {
                        s_hw[slot] = w;
                        s_hu[slot] = U;
                        s_hp[slot] = pw;
                        deferred = true;
                    }
                }
                for (uint32_t u0 = 0; !deferred && acc != U && u0 < nsym; u0 += SYM_BATCH) {
                    uint32_t beg[SYM_BATCH], end[SYM_BATCH];
                    if (u0 == 0) {
#pragma unroll
                        for (int j = 0; j < SYM_BATCH; j++) {
                            beg[j] = beg0[j];
                            end[j] = end0[j];
                        }
                    } else {
                        pull_rows<W>(p, w, U & ~acc, u0, beg, end);
                    }
#pragma unroll
                    for (int j = 0; j < SYM_BATCH; j++) {
                        uint32_t pj = end[j] > beg[j] ? succ_of(qv.pred, u0 + j, U & ~acc) : 0u;
                        for (uint32_t e = beg[j]; pj && e < end[j]; e++) {
                            const uint32_t m = ld_state<W>(Mc, g.col[e]) & pj;
                            if (m) {
                                acc |= succ_of(qv.succ, u0 + j, m) & U;
                                pj = succ_of(qv.pred, u0 + j, U & ~acc);
                            }
                        }
                    }
                }
                if (acc) st_state<W>(Mn, w, acc);  // only unvisited states: the next select adds them to P
            }
        }
        if (!block_append(acc != 0, static_cast<int32_t>(w), qn, &RN.nq, V)) flag_violation(p);
    }
    __syncthreads();
    // heavy vertices of this workgroup: one wavefront each, 64 neighbours per step
    const uint32_t nheavy = min(*s_hn, PULL_HEAVY_CAP);
    const uint32_t wave = threadIdx.x >> 6, nwaves = BLOCK / 64;
    for (uint32_t k = wave; k < nheavy; k += nwaves) {
        const uint32_t w = s_hw[k], U = s_hu[k], pw = s_hp[k];
        uint32_t acc = 0;
        for (uint32_t u = 0; u < nsym && acc != U; u++) {
            uint32_t pj = succ_of(qv.pred, u, U & ~acc);
            if (!pj) continue;
            const RankWordD rw = g.rankw[qv.pull_w[u] + (w >> 6)];
            uint32_t beg, end;
            if (!row_range(g, rw, qv.pull_r[u], w, beg, end)) continue;
            if (end > g.ncol || end < beg) {
                flag_violation(p);
                continue;
            }
            for (uint32_t e0 = beg; pj && e0 < end; e0 += 64) {
                const uint32_t e = e0 + lane;
                uint32_t got = 0;
                if (e < end) {
                    const uint32_t m = ld_state<W>(Mc, g.col[e]) & pj;
                    if (m) got = succ_of(qv.succ, u, m) & U;
                }
                acc |= wave_or(got);
                pj = succ_of(qv.pred, u, U & ~acc);
            }
        }
        if (lane == 0 && acc) {
            st_state<W>(Mn, w, acc);
            const uint32_t pos = atomicAdd(&RN.nq, 1u);
            if (pos < V) qn[pos] = static_cast<int32_t>(w);
            else flag_violation(p);
        }
        (void)pw;
    }
}

// After nlev levels: the result bitmap (vertex v has a final state: the
// product F P of Alg. 1) and P reset for the next query. The last level's
// words in M are cleared here only when that level pulled (clear_last); a push
// level has cleared them itself.
template <int W>
__device__ __forceinline__ void final_phase(const Params &p, uint32_t nlev, bool clear_last) {
    const uint32_t V = static_cast<uint32_t>(p.g.V);
    if (blockIdx.x == 0 && threadIdx.x == 0 && nlev < LVL_COUNT_CAP)
        p.st.lvl[static_cast<uint64_t>(nlev) * LVL_STRIDE + 3] = wall_clock64();
    // eight words of P per wave and step, all loaded before any is stored
    const uint32_t fm = s_qv.h->fmask;
    const uint32_t nwords = (V + 63) / 64;
    const uint32_t lane = lane_id();
    const uint32_t gw = gthread() >> 6, nw = gthreads() >> 6;
    for (uint32_t k0 = gw; k0 < nwords; k0 += 8 * nw) {
        uint32_t pv[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const uint32_t k = k0 + j * nw;
            const uint32_t v = k * 64 + lane;
            pv[j] = (k < nwords && v < V) ? ld_state<W>(p.st.P, v) : 0u;
        }
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const uint32_t k = k0 + j * nw;  // the same in the whole wave
            const uint64_t b = __ballot((pv[j] & fm) != 0);
            if (k < nwords) {
                if (lane == 0) p.st.out[k] = b;
                if (pv[j]) st_state<W>(p.st.P, k * 64 + lane, 0);
                // no accepted walk reaches v: its length is -1 (the others
                // were written by the select of their first final level)
                if (p.dist && !(pv[j] & fm) && k * 64 + lane < V) p.dist[k * 64 + lane] = -1;
            }
        }
    }
    if (nlev >= 1 && clear_last) {
        const uint32_t D = nlev - 1;
        const uint32_t nq = ld_acq(&p.st.rec[D % REC_RING].nq);
        uint32_t *M = p.st.M[D & 1];
        const int32_t *q = p.st.q[D & 1];
        for (uint32_t i = gthread(); i < nq; i += gthreads()) {
            const uint32_t v = static_cast<uint32_t>(ldc(&q[i]));
            if (v < V) st_state<W>(M, v, 0);
            else flag_violation(p);
        }
    }
}

// ------------------------------------------------------------ small levels
// A level with a short queue and few push edges is mostly fixed cost: two
// grid barriers (about 6 us each) and two dependent chains of loads. Such
// levels run in workgroup 0 alone, one after the other, with workgroup
// barriers in place of grid barriers, while the other workgroups wait at a
// single grid barrier. The phases and every array they touch are the same as
// in the grid-wide loop; all waves of workgroup 0 share one compute unit, so
// a workgroup barrier orders their memory accesses.
__device__ __forceinline__ void solo_sync() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Runs levels n, n+1, ... (level n's queue holds nq entries) in workgroup 0
// while they are small. Leaves in bar->solo_n the first level not finished,
// and in bar->solo_sel whether its select phase is already done (it was too
// large to push here, or the direction switch chose pull). The level records,
// the global queues and the item arrays are kept up to date as well, for the
// grid to take over from.
template <int W>
__device__ __forceinline__ void solo_levels(const Params &p, uint32_t n, uint32_t nq, uint32_t *s_eb,
                                            uint32_t *s_beg, uint32_t *s_mask, uint32_t &npush, uint64_t &tpairs) {
    __shared__ SoloLds so;
    uint32_t sel_done = 0;
    bool lq = false;  // level n's queue is in so.q (every level of the run but the first)
    for (uint32_t run = 0; run < SOLO_MAX_RUN; run++) {
        if (nq == 0 || nq > SOLO_MAX_QUEUE) break;
        select_phase<W, true>(p, n, nq, 0, 1, &so, lq, s_eb, s_beg, s_mask);
        // the stores to P and M are complete before the push loads P; the
        // items and totals are in LDS
        solo_sync();
        LevelInfo li;
        li.sel = so.sel;
        li.pairs = so.pairs;
        li.nfront = so.nfront;
        li.nq = nq;
        li.prev_mode = so.prev_mode;
        const uint32_t mode = decide(p, li);
        const uint32_t T = static_cast<uint32_t>(li.sel), nitems = static_cast<uint32_t>(li.sel >> 32);
        if (mode != 0 || T > SOLO_MAX_EDGES || nitems > static_cast<uint32_t>(TILE)) {
            sel_done = 1;
            break;
        }
        if (threadIdx.x == 0) record_level(p, n, 0, li);
        tpairs += li.pairs;
        // as push_phase: this level's words first, then the items' edges
        if (lq) clear_level_words<W, true>(p, n, nq, 0, 1, so.q[n & 1]);
        else clear_level_words<W>(p, n, nq, 0, 1);
        uint32_t nn = 0;
        if (T && nitems) nn = push_range<W, true>(p, n, s_eb, s_beg, s_mask, nitems, 0, T, so.q[(n + 1) & 1]);
        if (threadIdx.x == 0) p.st.rec[(n + 1) % REC_RING].nq = nn;
        __syncthreads();  // level n+1's queue is complete in LDS; the item copies are free
        npush++;
        n++;
        nq = nn;
        lq = true;
    }
    solo_sync();
    if (threadIdx.x == 0) {
        p.st.bar->solo_n = n;
        p.st.bar->solo_sel = sel_done;
    }
}

// ---------------------------------------------------------------- kernels
// A workgroup leaving the persistent kernel because a barrier timed out
// tells the host so.
__device__ __forceinline__ void leave_aborted(const Params &p) {
    if (threadIdx.x == 0) hstat_store(p, 6, 1u);
}

template <int W>
__global__ __launch_bounds__(BLOCK) void k_persistent(Params p) {
    // push tiles and pull heavy lists share the workgroup's LDS
    __shared__ uint32_t s_eb[TILE + 1], s_beg[TILE + 1], s_mask[TILE + 1], s_hn;
    qv_setup<true>(p.qv);
    GridBarrier *bar = p.st.bar;
    // the next launch's barrier (not touched by this one) starts zeroed: no
    // separate clearing launch per query
    if (blockIdx.x == 0 && p.st.bar_next) {
        uint32_t *z = reinterpret_cast<uint32_t *>(p.st.bar_next);
        for (uint32_t i = threadIdx.x; i < sizeof(GridBarrier) / 4; i += BLOCK) z[i] = 0;
    }
    barrier_arrive_register(bar);
    uint32_t n = 0, npush = 0, npull = 0, last_mode = 0;
    uint64_t tpairs = 0;  // |P|, summed over the levels (workgroup 0's count is complete)
    // Level 0's queue is known without reading memory: M_0 = Q_S x {source},
    // one entry (none without start states). Workgroup 0 initialises the query
    // and runs the first small levels while the rest of the grid is still
    // being dispatched and registering; the others wait at the first barrier.
    if (blockIdx.x == 0) {
        init_phase<W>(p);
        solo_sync();  // level 0's queue and words are in memory before the run reads them
        const uint32_t nq0 = s_qv.h->smask ? (p.nsrc ? p.nsrc : 1u) : 0u;
        solo_levels<W>(p, 0, nq0, s_eb, s_beg, s_mask, npush, tpairs);
    }
    BarCtx bc;
    if (!barrier_wait_register(bar, bc)) return leave_aborted(p);
    if (!grid_barrier(bar, bc)) return leave_aborted(p);
    n = ld_acq(&bar->solo_n);
    bool selected = ld_acq(&bar->solo_sel) != 0;  // level n's select is done
    uint32_t solo_at = 0;
    uint32_t nq_known = ~0u;  // level n's queue length when already loaded
    while (true) {
        if (!selected) {
            const uint32_t nq = nq_known != ~0u ? nq_known : ld_acq(&p.st.rec[n % REC_RING].nq);
            nq_known = ~0u;
            if (nq == 0) break;
            if (nq <= SOLO_MAX_QUEUE && n != solo_at) {
                // a run of small levels in workgroup 0; the rest wait here
                solo_at = n;
                if (blockIdx.x == 0) solo_levels<W>(p, n, nq, s_eb, s_beg, s_mask, npush, tpairs);
                if (!grid_barrier(bar, bc)) return leave_aborted(p);
                n = ld_acq(&bar->solo_n);
                selected = ld_acq(&bar->solo_sel) != 0;
                last_mode = 0;  // solo levels push (a level it left selected is expanded next)
                continue;
            }
            if (last_mode == 0 && s_qv.h->force != 2 && nq <= static_cast<uint32_t>(p.g.V) / FUSE_V_DIV) {
                // a fused level: select and push of each workgroup's own items,
                // then one barrier (and a grid-wide push of what exceeded the
                // workgroups' budgets, if anything did)
                select_phase<W, false, true>(p, n, nq, blockIdx.x, gridDim.x, nullptr, false, s_eb, s_beg, s_mask);
                if (!grid_barrier(bar, bc)) return leave_aborted(p);
                const LevelInfo li = level_info(p, n);  // sel: the global items only
                // the next queue's length, loaded with the totals (final
                // unless the grid push below still appends)
                const uint32_t nq_next = ld_acq(&p.st.rec[(n + 1) % REC_RING].nq);
                if (blockIdx.x == 0 && threadIdx.x == 0) {
                    LevelInfo all = li;
                    all.sel += ld_acq(&p.st.rec[n % REC_RING].hsel);
                    record_level(p, n, 0, all);
                }
                tpairs += li.pairs;
                if (li.sel >> 32) {
                    push_phase<W>(p, n, li, s_eb, s_beg, s_mask, blockIdx.x, gridDim.x, false);
                    if (!grid_barrier(bar, bc)) return leave_aborted(p);
                } else {
                    nq_known = nq_next;
                }
                npush++;
                last_mode = 0;
                n++;
                continue;
            }
            select_phase<W>(p, n, nq, blockIdx.x, gridDim.x);
            if (!grid_barrier(bar, bc)) return leave_aborted(p);
        }
        selected = false;
        const LevelInfo li = level_info(p, n);
        const uint32_t mode = decide(p, li);
        if (blockIdx.x == 0 && threadIdx.x == 0) record_level(p, n, mode, li);
        tpairs += li.pairs;
        if (mode == 0) push_phase<W>(p, n, li, s_eb, s_beg, s_mask, blockIdx.x, gridDim.x);
        else pull_phase<W>(p, n, s_eb, s_beg, s_mask, &s_hn);
        npush += mode == 0;
        npull += mode != 0;
        last_mode = mode;
        if (!grid_barrier(bar, bc)) return leave_aborted(p);
        n++;
    }
    final_phase<W>(p, n, last_mode != 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // A fused level's pushes may read P before other workgroups' selects
        // of the same level add to it, so its candidates may turn out to hold
        // only visited states: the next frontier is then empty and yields no
        // items, which makes it the last level. It is not counted.
        if (n >= 1 && ld_acq(&p.st.rec[(n - 1) % REC_RING].pairs) == 0) {
            n--;
            if (last_mode == 0) npush--;
            else npull--;
        }
        p.st.status[0] = n;
        p.st.status[1] = npush;
        p.st.status[2] = npull;
        p.st.status[4] = static_cast<uint32_t>(tpairs);
        p.st.status[5] = static_cast<uint32_t>(tpairs >> 32);
        // the same words for the host, and the launch's serial last
        hstat_store(p, 0, n);
        hstat_store(p, 1, npush);
        hstat_store(p, 2, npull);
        hstat_store(p, 4, static_cast<uint32_t>(tpairs));
        hstat_store(p, 5, static_cast<uint32_t>(tpairs >> 32));
        hstat_store(p, 7, p.st.hserial);
    }
}

template <int W>
__global__ __launch_bounds__(64) void k_init(Params p) {
    qv_setup<false>(p.qv);
    init_phase<W>(p);
}

template <int W>
__global__ __launch_bounds__(BLOCK) void k_select(Params p, uint32_t n) {
    qv_setup<false>(p.qv);
    select_phase<W>(p, n, ld_acq(&p.st.rec[n % REC_RING].nq), blockIdx.x, gridDim.x);
}

template <int W>
__global__ __launch_bounds__(BLOCK) void k_expand(Params p, uint32_t n) {
    __shared__ uint32_t s_eb[TILE + 1], s_beg[TILE + 1], s_mask[TILE + 1], s_hn;
    qv_setup<false>(p.qv);
    const LevelInfo li = level_info(p, n);
    const uint32_t mode = decide(p, li);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        record_level(p, n, mode, li);
        p.st.status[0] = n + 1;
        p.st.status[1 + (mode != 0)] += 1;
    }
    if (mode == 0) push_phase<W>(p, n, li, s_eb, s_beg, s_mask, blockIdx.x, gridDim.x);
    else pull_phase<W>(p, n, s_eb, s_beg, s_mask, &s_hn);
}

// Levels in a captured graph: the same phases as k_select / k_expand, with
// the Params block in device memory (one graph serves every query of the
// handle) and the level number in gctl, advanced on the device; once a level
// ends the traversal, the later nodes of the replay return at once. The done
// flag only changes between kernels, so each workgroup reads one value.
template <int W>
__global__ __launch_bounds__(BLOCK) void k_select_g(const Params *pp) {
    const Params &p = *pp;
    if (ld_acq(&p.st.gctl[1])) return;
    qv_setup<false>(p.qv);
    const uint32_t n = ld_acq(&p.st.gctl[0]);
    select_phase<W>(p, n, ld_acq(&p.st.rec[n % REC_RING].nq), blockIdx.x, gridDim.x);
}

template <int W>
__global__ __launch_bounds__(BLOCK) void k_expand_g(const Params *pp) {
    __shared__ uint32_t s_eb[TILE + 1], s_beg[TILE + 1], s_mask[TILE + 1], s_hn;
    const Params &p = *pp;
    if (ld_acq(&p.st.gctl[1])) return;
    qv_setup<false>(p.qv);
    const uint32_t n = ld_acq(&p.st.gctl[0]);
    const LevelInfo li = level_info(p, n);
    const uint32_t mode = decide(p, li);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        record_level(p, n, mode, li);
        p.st.status[0] = n + 1;
        p.st.status[1 + (mode != 0)] += 1;
    }
    if (mode == 0) push_phase<W>(p, n, li, s_eb, s_beg, s_mask, blockIdx.x, gridDim.x);
    else pull_phase<W>(p, n, s_eb, s_beg, s_mask, &s_hn);
}

__global__ void k_advance_g(const Params *pp) {
    const Params &p = *pp;
    if (threadIdx.x != 0 || ld_acq(&p.st.gctl[1])) return;
    const uint32_t n = ld_acq(&p.st.gctl[0]);
    if (ld_acq(&p.st.rec[(n + 1) % REC_RING].nq) == 0) {
        p.st.gctl[2] = n + 1;
        p.st.gctl[1] = 1;
    } else {
        p.st.gctl[0] = n + 1;
    }
}

template <int W>
__global__ __launch_bounds__(BLOCK) void k_final(Params p, uint32_t nlev) {
    qv_setup<false>(p.qv);
    final_phase<W>(p, nlev, nlev >= 1 && ld_acq(&p.st.rec[(nlev - 1) % REC_RING].mode) != 0);
}

__global__ void k_fill(uint32_t *ptr, uint64_t words, uint32_t value) {
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        ptr[i] = value;
}

// ---------------------------------------------------------------- launchers
// The grid (persistent_grid) is at most one workgroup per CU and fits the
// occupancy limit, so on an idle GPU every workgroup is resident at once; an
// ordinary launch dispatches about 14 us faster than a cooperative one. A
// workgroup held back by other work longer than the barrier's time-out makes
// the launch abort (status word), never wait for good.
template <int W>
static hipError_t launch_persistent_w(const Params &p, int grid, bool cooperative, hipStream_t s) {
    Params a = p;
    if (cooperative) {
        void *args[] = {&a};
        return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_persistent<W>), dim3(grid),
                                          dim3(BLOCK), args, 0, s);
    }
    hipLaunchKernelGGL(k_persistent<W>, dim3(grid), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_persistent(int W, const Params &p, int grid, bool cooperative, hipStream_t s) {
    switch (W) {
        case 1: return launch_persistent_w<1>(p, grid, cooperative, s);
        case 2: return launch_persistent_w<2>(p, grid, cooperative, s);
        default: return launch_persistent_w<4>(p, grid, cooperative, s);
    }
}

int occupancy_blocks_per_cu(int W) {
    int per = 0;
    hipError_t e;
    switch (W) {
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<1>, BLOCK, 0); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<2>, BLOCK, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<4>, BLOCK, 0); break;
    }
    return e == hipSuccess ? per : -1;
}

int persistent_grid(int W) {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e;
    switch (W) {
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<1>, BLOCK, 0); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<2>, BLOCK, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<4>, BLOCK, 0); break;
    }
    if (e != hipSuccess || per < 1) return 0;
    return ncu * (per < PERSISTENT_BLOCKS_PER_CU ? per : PERSISTENT_BLOCKS_PER_CU);
}

#define RPQ_DISPATCH_W(W, CALL) \
    switch (W) {                \
        case 1: { constexpr int WW = 1; CALL; } break; \
        case 2: { constexpr int WW = 2; CALL; } break; \
        default: { constexpr int WW = 4; CALL; } break; \
    }

hipError_t launch_init(int W, const Params &p, hipStream_t s) {
    RPQ_DISPATCH_W(W, hipLaunchKernelGGL(k_init<WW>, dim3(1), dim3(64), 0, s, p));
    return hipGetLastError();
}

hipError_t launch_level_g(int W, const Params *pdev, int grid, hipStream_t s) {
    RPQ_DISPATCH_W(W, hipLaunchKernelGGL(k_select_g<WW>, dim3(grid), dim3(BLOCK), 0, s, pdev));
    RPQ_DISPATCH_W(W, hipLaunchKernelGGL(k_expand_g<WW>, dim3(grid), dim3(BLOCK), 0, s, pdev));
    hipLaunchKernelGGL(k_advance_g, dim3(1), dim3(64), 0, s, pdev);
    return hipGetLastError();
}

hipError_t launch_select(int W, const Params &p, uint32_t level, int grid, hipStream_t s) {
    RPQ_DISPATCH_W(W, hipLaunchKernelGGL(k_select<WW>, dim3(grid), dim3(BLOCK), 0, s, p, level));
    return hipGetLastError();
}

hipError_t launch_expand(int W, const Params &p, uint32_t level, int grid, hipStream_t s) {
    RPQ_DISPATCH_W(W, hipLaunchKernelGGL(k_expand<WW>, dim3(grid), dim3(BLOCK), 0, s, p, level));
    return hipGetLastError();
}

hipError_t launch_final(int W, const Params &p, uint32_t nlevels, int grid, hipStream_t s) {
    RPQ_DISPATCH_W(W, hipLaunchKernelGGL(k_final<WW>, dim3(grid), dim3(BLOCK), 0, s, p, nlevels));
    return hipGetLastError();
}

hipError_t launch_fill(uint32_t *ptr, uint64_t words, uint32_t value, hipStream_t s) {
    if (words == 0) return hipSuccess;
    uint64_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, ptr, words, value);
    return hipGetLastError();
}

}  // namespace rpq
