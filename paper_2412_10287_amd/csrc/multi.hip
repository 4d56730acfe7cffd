// Multi-query kernels: every admitted query (a slot, with its own NFA, source,
// visited set P and frontier M) advances one level per launch pair. The level
// is the same computation as the single-query path (Alg. 1's update: for each
// frontier pair set, succ_a per used symbol, pushed along the symbol's rows,
// masked by P, the mask applied to the candidates in the next select), with a
// slot tag on every queue entry and push item, so one edge-balanced launch
// carries the frontiers of all queries at once and the per-level fixed cost
// is shared.
#include "device_common.h"
#include "multi.h"

namespace rpq {

__device__ __forceinline__ void mviolation(const MultiParams &p) { atomicAdd(p.status, 1u); }

// Tables of slot s (same layout as build_qconst).
__device__ __forceinline__ QueryView slot_view(const MultiParams &p, uint32_t s) {
    const uint8_t *base = p.qconst + static_cast<size_t>(s) * QC_STRIDE;
    return qconst_view(base, reinterpret_cast<const QHeader *>(base)->nsym);
}

// One workgroup per admitted request: its query constants from the staging
// upload into the slot's block, then the start pairs.
__global__ void k_multi_admit(MultiParams p, uint32_t parity, uint32_t n, const uint8_t *stage) {
    const uint32_t i = blockIdx.x;
    if (i >= n) return;
    const uint32_t *rec = reinterpret_cast<const uint32_t *>(stage) + 4 * i;
    const uint32_t s = rec[0], v = rec[1], off = rec[2], bytes = rec[3];
    if (s >= p.slots || v >= static_cast<uint32_t>(p.V) || bytes < sizeof(QHeader) || bytes > QC_STRIDE ||
        off % 16 != 0 || off < ADMIT_TABLE_BYTES || off > ADMIT_TABLE_BYTES + QC_STRIDE * p.slots - bytes) {
        if (threadIdx.x == 0) mviolation(p);
        return;
    }
    const uint4 *src = reinterpret_cast<const uint4 *>(stage + off);
    uint4 *dst = reinterpret_cast<uint4 *>(const_cast<uint8_t *>(p.qconst) + static_cast<size_t>(s) * QC_STRIDE);
    for (uint32_t k = threadIdx.x; k < (bytes + 15) / 16; k += blockDim.x) dst[k] = src[k];
    if (threadIdx.x != 0) return;
    const uint32_t sm = reinterpret_cast<const QHeader *>(stage + off)->smask;
    p.pairs[s * PAIRS_STRIDE] = 0;
    p.dead[s] = 0;
    if (!sm) return;
    // M_0 = Q_S x {source} as a candidate: the next select adds it to P
    p.M[parity][s * p.swords + v] = sm;
    const uint32_t pos = atomicAdd(p.qlen[parity], 1u);
    if (pos < p.queue_cap) p.q[parity][pos] = (s << p.vbits) | v;
    else mviolation(p);
}

// Queue entries [lo, hi) of the current level -> items. The first chunk of a
// level also clears the previous level's frontier words (the buffer this level
// writes) and resets the per-slot append counters and the next queue length.
__global__ __launch_bounds__(BLOCK) void k_multi_select(MultiParams p, uint32_t parity, uint32_t lo, uint32_t hi,
                                                        uint32_t clear_n, int first_chunk, uint32_t chunk_id) {
    const uint32_t V = static_cast<uint32_t>(p.V);
    const uint32_t vmask = (1u << p.vbits) - 1u;
    uint64_t *sel = p.sel + (chunk_id & 1);
    // reached pairs per slot, summed in LDS and added to the slot counters
    // once per workgroup
    __shared__ unsigned long long s_pairs[MAX_SLOTS_DEV];
    for (uint32_t i = threadIdx.x; i < MAX_SLOTS_DEV; i += BLOCK) s_pairs[i] = 0;
    __syncthreads();
    // the other reservation counter was read by the previous push, which has
    // finished: clear it for the next chunk
    if (gthread() == 0) p.sel[(chunk_id + 1) & 1] = 0;
    if (first_chunk) {
        uint32_t *Mold = p.M[parity ^ 1];
        const uint32_t *qold = p.q[parity ^ 1];
        for (uint32_t i = gthread(); i < clear_n; i += gthreads()) {
            const uint32_t e = qold[i], s = e >> p.vbits, v = e & vmask;
            if (s < p.slots && v < V) Mold[s * p.swords + v] = 0;
            else mviolation(p);
        }
        for (uint32_t i = gthread(); i < p.slots; i += gthreads()) p.next_count[i] = 0;
        if (gthread() == 0) *p.qlen[parity ^ 1] = 0;
    }
    const uint32_t *qc = p.q[parity];
    uint32_t *Mc = p.M[parity];
    const GraphView &g = p.g;
    // workgroup-uniform loop: item reservations are made per workgroup
    for (uint32_t bbase = lo + blockIdx.x * BLOCK; bbase < hi; bbase += gridDim.x * BLOCK) {
        const uint32_t i = bbase + threadIdx.x;
        uint32_t s = 0, v = 0, S = 0, nsym = 0;
        QueryView qv{};
        if (i < hi) {
            const uint32_t e = qc[i];
            s = e >> p.vbits;
            v = e & vmask;
            if (s < p.slots && v < V) {
                // the complement mask of Alg. 1, then P = P + M
                const uint64_t at = s * p.swords + v;
                const uint32_t c = Mc[at];
                const uint32_t pv = p.P[at];
                // a slot whose query moved to a lane: its candidates are
                // dropped, so its frontier ends here
                S = p.dead[s] ? 0u : (c & ~pv);
                if (S) p.P[at] = pv | S;
                if (S != c) Mc[at] = S;
                qv = slot_view(p, s);
                nsym = qv.h->nsym;
            } else {
                mviolation(p);
                s = v = 0;
            }
        }
        if (S) atomicAdd(&s_pairs[s < MAX_SLOTS_DEV ? s : 0], static_cast<unsigned long long>(__popc(S)));
        // only the symbols with a transition out of S can give an item; the
        // rounds continue while any lane of the workgroup has symbols left
        SymSet Rs = symbols_of(qv, S, nsym);
        while (true) {
            uint32_t us[SYM_BATCH], sp[SYM_BATCH], beg[SYM_BATCH], len[SYM_BATCH];
            RankWordD rw[SYM_BATCH];
#pragma unroll
            for (int j = 0; j < SYM_BATCH; j++) us[j] = symbol_pop(Rs);
            bool more = false;
#pragma unroll
            for (int k = 0; k < SYM_WORDS; k++) more = more || Rs.w[k] != 0;
#pragma unroll
            for (int j = 0; j < SYM_BATCH; j++) {
                sp[j] = us[j] < nsym ? succ_of(qv.succ, us[j], S) : 0u;
                if (sp[j]) rw[j] = g.rankw[qv.push_w[us[j]] + (v >> 6)];
            }
            uint32_t cnt = 0, tot = 0;
#pragma unroll
            for (int j = 0; j < SYM_BATCH; j++) {
                len[j] = 0;
                uint32_t e;
                if (sp[j] && row_range(g, rw[j], qv.push_r[us[j]], v, beg[j], e)) {
                    if (e > beg[j] && e <= g.ncol) len[j] = e - beg[j];
                    else if (e != beg[j]) mviolation(p);
                }
                if (len[j]) {
                    cnt++;
                    tot += len[j];
                }
            }
            uint64_t wtot;
            const uint64_t ex = wave_excl_scan((static_cast<uint64_t>(cnt) << SEL_SHIFT) | tot, wtot);
            uint64_t wbase;
            const bool bmore = block_reserve<uint64_t>(wtot, more, sel, wbase);
            if (cnt) {
                const uint64_t mine = wbase + ex;
                uint64_t idx = mine >> SEL_SHIFT;
                uint64_t eb = mine & ((1ull << SEL_SHIFT) - 1);
#pragma unroll
                for (int j = 0; j < SYM_BATCH; j++) {
                    if (!len[j]) continue;
                    if (idx < p.item_cap) {
                        p.it_ebase[idx] = eb;
                        p.it_beg[idx] = beg[j];
                        p.it_mask[idx] = sp[j];
                        p.it_slot[idx] = s;
                    } else {
                        mviolation(p);
                    }
                    const uint64_t k1 = (eb + len[j] - 1) / TILE;
                    for (uint64_t k = (eb + TILE - 1) / TILE; k <= k1; k++) {
                        if (k < p.tile_cap) p.tile_first[k] = static_cast<uint32_t>(idx);
                        else { mviolation(p); break; }
                    }
                    idx++;
                    eb += len[j];
                }
            }
            if (!bmore) break;
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < p.slots && i < MAX_SLOTS_DEV; i += BLOCK)
        if (s_pairs[i]) atomicAdd(reinterpret_cast<unsigned long long *>(&p.pairs[i * PAIRS_STRIDE]), s_pairs[i]);
}

// Edges [ubase, uend) of the items staged in LDS (cnt of them), four per
// thread and step: the loads of col and P for all four, then the atomics,
// then one queue reservation per workgroup. The states of an item not yet in P[w]
// are ORed into w's next word; the first writer appends (slot, w).
__device__ __forceinline__ void multi_push_range(const MultiParams &p, uint32_t parity, const uint64_t *s_eb,
                                                 const uint32_t *s_beg, const uint32_t *s_mask, const uint32_t *s_slot,
                                                 uint32_t cnt, uint64_t ubase, uint64_t uend) {
    const uint32_t V = static_cast<uint32_t>(p.V);
    uint32_t *qn = p.q[parity ^ 1];
    uint32_t *Mn = p.M[parity ^ 1];
    const uint32_t *col = p.g.col;
    const uint32_t tid = threadIdx.x;
    static_assert(TILE == 4 * BLOCK, "four edges per thread and step");
    // the halving steps of the item search depend on cnt alone (the same in
    // every lane): a uniform loop of ceil(log2(cnt)) steps, no step for one item
    const uint32_t ucnt = __builtin_amdgcn_readfirstlane(cnt);
    for (uint64_t ub = ubase; ub < uend; ub += TILE) {
        uint32_t w[4], sp[4], sl[4], lo[4];
        uint64_t tt[4];
        // last staged item with s_eb <= t (s_eb[0] <= ubase); lanes past
        // uend search for uend - 1 and drop the result
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint64_t t = ub + static_cast<uint64_t>(k) * BLOCK + tid;
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
            const uint64_t t = ub + static_cast<uint64_t>(k) * BLOCK + tid;
            w[k] = V;
            sp[k] = 0;
            sl[k] = 0;
            if (t < uend) {
                const uint64_t pos = s_beg[lo[k]] + (t - s_eb[lo[k]]);
                sp[k] = s_mask[lo[k]];
                sl[k] = s_slot[lo[k]];
                if (pos < p.g.ncol && sl[k] < p.slots) {
                    w[k] = col[pos];
                    if (w[k] >= V) {
                        mviolation(p);
                        w[k] = V;
                    }
                } else {
                    mviolation(p);
                }
            }
        }
        uint32_t cand[4];
#pragma unroll
        for (int k = 0; k < 4; k++) cand[k] = w[k] < V ? sp[k] & ~p.P[sl[k] * p.swords + w[k]] : 0u;
        bool first[4];
#pragma unroll
        for (int k = 0; k < 4; k++) first[k] = cand[k] ? atomicOr(&Mn[sl[k] * p.swords + w[k]], cand[k]) == 0u : false;
        if (!block_append4(first[0], static_cast<int32_t>((sl[0] << p.vbits) | w[0]), first[1],
                           static_cast<int32_t>((sl[1] << p.vbits) | w[1]), first[2],
                           static_cast<int32_t>((sl[2] << p.vbits) | w[2]), first[3],
                           static_cast<int32_t>((sl[3] << p.vbits) | w[3]), reinterpret_cast<int32_t *>(qn),
                           p.qlen[parity ^ 1], static_cast<uint32_t>(p.queue_cap)))
            mviolation(p);
        // the host only asks whether a slot still has a frontier: a plain
        // store of 1 (every writer stores the same value), skipped once this
        // XCD's copy of the flag reads 1
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (first[k] && p.next_count[sl[k]] == 0u) p.next_count[sl[k]] = 1u;
    }
}

// Items -> edges, spread evenly over the grid: with few items every workgroup
// stages all of them and takes an even, wave-aligned share of the edges;
// otherwise tiles of TILE edges (split into parts when there are fewer tiles
// than workgroups) stage their own items.
__global__ __launch_bounds__(BLOCK) void k_multi_push(MultiParams p, uint32_t parity, uint32_t chunk_id) {
    __shared__ uint64_t s_eb[TILE + 1];
    __shared__ uint32_t s_beg[TILE + 1], s_mask[TILE + 1], s_slot[TILE + 1];
    const uint64_t sel = __hip_atomic_load(p.sel + (chunk_id & 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t nitems = sel >> SEL_SHIFT;
    const uint64_t T = sel & ((1ull << SEL_SHIFT) - 1);
    if (T == 0 || nitems == 0) return;
    const uint64_t ntiles = (T + TILE - 1) / TILE;
    if (nitems > p.item_cap || ntiles > p.tile_cap) {
        if (gthread() == 0) mviolation(p);
        return;
    }
    const uint32_t tid = threadIdx.x;
    if (nitems <= static_cast<uint64_t>(TILE)) {
        for (uint32_t j = tid; j < nitems; j += BLOCK) {
            s_eb[j] = p.it_ebase[j];
            s_beg[j] = p.it_beg[j];
            s_mask[j] = p.it_mask[j];
            s_slot[j] = p.it_slot[j];
        }
        __syncthreads();
        uint64_t per = (T + gridDim.x - 1) / gridDim.x;
        per = (per + 63) & ~63ull;
        const uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * per;
        const uint64_t b1 = b0 + per < T ? b0 + per : T;
        if (b0 < b1) multi_push_range(p, parity, s_eb, s_beg, s_mask, s_slot, static_cast<uint32_t>(nitems), b0, b1);
        return;
    }
    uint32_t sub = 1;
    while (sub < TILE / 64 && ntiles * sub * 2 <= gridDim.x) sub *= 2;
    const uint32_t part = TILE / sub;
    for (uint64_t vt = blockIdx.x; vt < ntiles * sub; vt += gridDim.x) {
        const uint64_t tile = vt / sub;
        const uint32_t k = static_cast<uint32_t>(vt % sub);
        uint32_t i0 = p.tile_first[tile];
        uint32_t i1 = tile + 1 < ntiles ? p.tile_first[tile + 1] : static_cast<uint32_t>(nitems - 1);
        if (i0 >= nitems || i1 >= nitems || i1 < i0 || i1 - i0 > static_cast<uint32_t>(TILE)) {
            if (tid == 0) mviolation(p);
            i0 = i1 = 0;
        }
        const uint32_t cnt = i1 - i0 + 1;
        for (uint32_t j = tid; j < cnt; j += BLOCK) {
            s_eb[j] = p.it_ebase[i0 + j];
            s_beg[j] = p.it_beg[i0 + j];
            s_mask[j] = p.it_mask[i0 + j];
            s_slot[j] = p.it_slot[i0 + j];
        }
        __syncthreads();
        const uint64_t u0 = tile * TILE + static_cast<uint64_t>(k) * part;
        const uint64_t u1 = u0 + part < T ? u0 + part : T;
        if (u0 < u1) multi_push_range(p, parity, s_eb, s_beg, s_mask, s_slot, cnt, u0, u1);
        __syncthreads();
    }
}

// One wavefront per 64-vertex word of each finished slot's answer: the ballot
// of (P[v] & F != 0) is the word (the product F P of Alg. 1); P is reset.
// fin holds (slot, result-pool entry) pairs.
__global__ __launch_bounds__(BLOCK) void k_multi_extract(MultiParams p, FinList fin, uint64_t nwords) {
    const uint32_t V = static_cast<uint32_t>(p.V);
    const uint32_t lane = lane_id();
    const uint32_t nfin = fin.n <= MAX_SLOTS_DEV ? fin.n : MAX_SLOTS_DEV;
    const uint64_t total = static_cast<uint64_t>(nfin) * nwords;
    for (uint64_t gw = gthread() >> 6; gw < total; gw += gthreads() >> 6) {
        const uint32_t f = static_cast<uint32_t>(gw / nwords);
        const uint64_t k = gw % nwords;
        const uint32_t s = fin.e[2 * f], entry = fin.e[2 * f + 1];
        if (s >= p.slots || entry >= 3 * p.slots) {
            if (lane == 0) mviolation(p);
            continue;
        }
        const uint32_t fm = reinterpret_cast<const QHeader *>(p.qconst + static_cast<size_t>(s) * QC_STRIDE)->fmask;
        const uint64_t v = k * 64 + lane;
        uint32_t *Ps = p.P + static_cast<uint64_t>(s) * p.swords;
        const uint32_t pv = v < V ? Ps[v] : 0u;
        const uint64_t b = __ballot((pv & fm) != 0);
        if (lane == 0) p.out[static_cast<uint64_t>(entry) * nwords + k] = b;
        if (pv) Ps[v] = 0;
    }
}

hipError_t multi_admit(const MultiParams &p, uint32_t parity, uint32_t n, const uint8_t *stage, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_multi_admit, dim3(n), dim3(256), 0, s, p, parity, n, stage);
    return hipGetLastError();
}

// Device-scope loads of the block the level's kernels wrote, system-scope
// stores into the pinned host copy.
__global__ void k_multi_publish(const uint32_t *ctl, uint32_t *host, uint32_t words) {
    for (uint32_t i = threadIdx.x; i < words; i += blockDim.x)
        __hip_atomic_store(host + i, ldc(ctl + i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void k_copy_signal(const uint64_t *src, uint64_t *dst, uint64_t nwords, uint32_t *done, uint32_t *flag,
                              uint32_t seq) {
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nwords;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        dst[i] = src[i];
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores are in L2
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // system scope: the L2 is written back
        const uint32_t prev = __hip_atomic_fetch_add(done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_SYSTEM);
        if (prev == gridDim.x - 1) {
            __hip_atomic_store(done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

hipError_t copy_signal(const uint64_t *src, uint64_t *dst, uint64_t nwords, uint32_t *done, uint32_t *flag,
                       uint32_t seq, hipStream_t s) {
    uint64_t blocks = (nwords + 4095) / 4096;  // 1024 threads, 4 words each
    if (blocks < 1) blocks = 1;
    if (blocks > 64) blocks = 64;
    hipLaunchKernelGGL(k_copy_signal, dim3(static_cast<uint32_t>(blocks)), dim3(1024), 0, s, src, dst, nwords, done,
                       flag, seq);
    return hipGetLastError();
}

hipError_t multi_publish(const MultiParams &p, uint32_t *host, uint32_t words, hipStream_t s) {
    hipLaunchKernelGGL(k_multi_publish, dim3(1), dim3(1024), 0, s, p.ctl, host, words);
    return hipGetLastError();
}

hipError_t multi_select(const MultiParams &p, uint32_t parity, uint32_t lo, uint32_t hi, uint32_t clear_n,
                        int first_chunk, uint32_t chunk_id, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_multi_select, dim3(grid), dim3(BLOCK), 0, s, p, parity, lo, hi, clear_n, first_chunk,
                       chunk_id);
    return hipGetLastError();
}

hipError_t multi_push(const MultiParams &p, uint32_t parity, uint32_t chunk_id, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_multi_push, dim3(grid), dim3(BLOCK), 0, s, p, parity, chunk_id);
    return hipGetLastError();
}

hipError_t multi_extract(const MultiParams &p, const FinList &fin, uint64_t nwords, hipStream_t s) {
    if (!fin.n || fin.n > MAX_SLOTS_DEV) return fin.n ? hipErrorInvalidValue : hipSuccess;
    uint64_t waves = static_cast<uint64_t>(fin.n) * nwords;
    uint64_t blocks = (waves + (BLOCK / 64) - 1) / (BLOCK / 64);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_multi_extract, dim3(static_cast<uint32_t>(blocks)), dim3(BLOCK), 0, s, p, fin, nwords);
    return hipGetLastError();
}

}  // namespace rpq
