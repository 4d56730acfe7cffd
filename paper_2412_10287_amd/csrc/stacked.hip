// Stacked multi-source traversal (the multiple-source direction of Sec. 6):
// B sources under one NFA share one level-synchronous traversal. For every
// vertex v and state q, the frontier and visited sets hold a row of B source
// bits, so the level update of Alg. 1 becomes, per edge (v, w) of symbol a and
// transition q -a-> q',
//     new = M[v][q] AND NOT P[w][q'],   P[w][q'] |= new,   M'[w][q'] |= new
// on 64-bit words: one random access to w's row serves 64 sources per word
// (the bit-parallel multi-source BFS idea of Then et al., VLDB 2014).
//
// Phases per level (one cooperative launch, grid barriers between phases):
//   select  frontier vertex v with state support S(v) -> one item per used
//           symbol u with succ_u(S(v)) non-empty and a u-row at v;
//   push    edges of all items spread evenly, G lanes per edge (one 64-bit
//           word each), atomics fused with the not-P mask;
// and after the last level an extract phase that turns the per-vertex rows of
// final states into one result bitmap per source and resets P.
#include "device_common.h"
#include "stacked.h"

namespace rpq {

__device__ __forceinline__ void sviol(const StackParams &p) { atomicAdd(&p.status[3], 1u); }

template <int G>
__device__ __forceinline__ uint64_t row_index(const StackParams &p, uint32_t v, uint32_t q) {
    return (static_cast<uint64_t>(v) * static_cast<uint32_t>(p.Q) + q) * G;
}

template <int G>
__device__ void st_select(const StackParams &p, uint32_t n) {
    const GraphView &g = p.g;
    const QueryView &qv = p.qv;
    LevelRec *rec = p.rec;
    LevelRec &R = rec[n % REC_RING];
    const uint32_t nq = ld_acq(&R.nq);
    const uint32_t V = static_cast<uint32_t>(p.V);
    const uint32_t Q = static_cast<uint32_t>(p.Q);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rec[(n + 1) % REC_RING] = LevelRec{};
        if (n < LVL_COUNT_CAP) p.lvl_pairs[n] = static_cast<int64_t>(ld_acq(&R.pairs));
    }
    // rows of the previous frontier live in the buffer this level writes
    if (n >= 1) {
        const uint32_t nprev = ld_acq(&rec[(n - 1) % REC_RING].nq);
        uint64_t *Mold = p.M[(n + 1) & 1];
        uint32_t *sold = p.sup[(n + 1) & 1];
        const int32_t *qold = p.q[(n + 1) & 1];
        const uint64_t words = static_cast<uint64_t>(Q) * G;
        const uint64_t total = static_cast<uint64_t>(nprev) * words;
        for (uint64_t x = gthread(); x < total; x += gthreads()) {
            const uint32_t v = static_cast<uint32_t>(qold[x / words]);
            const uint32_t k = static_cast<uint32_t>(x % words);
            if (v >= V) {
                sviol(p);
                continue;
            }
            Mold[static_cast<uint64_t>(v) * words + k] = 0;
            if (k == 0) sold[v] = 0;
        }
    }
    const int32_t *qc = p.q[n & 1];
    const uint32_t *sc = p.sup[n & 1];
    const uint32_t lane = lane_id();
    const uint32_t gw = gthread() >> 6, nw = gthreads() >> 6;
    const uint32_t nsym = qv.h->nsym;
    constexpr uint32_t TE = TILE / G;  // edges per push tile
    for (uint32_t base = gw * 64; base < nq; base += nw * 64) {
        const uint32_t i = base + lane;
        uint32_t v = i < nq ? static_cast<uint32_t>(qc[i]) : 0u;
        uint32_t S = 0;
        if (i < nq) {
            if (v < V) S = sc[v];
            else { sviol(p); v = 0; }
        }
        for (uint32_t u0 = 0; u0 < nsym; u0 += SYM_BATCH) {
            uint32_t sp[SYM_BATCH], beg[SYM_BATCH], len[SYM_BATCH];
            RankWordD rw[SYM_BATCH];
#pragma unroll
            for (int j = 0; j < SYM_BATCH; j++) {
                const uint32_t u = u0 + j;
                sp[j] = (S && u < nsym) ? succ_of(qv.succ, u, S) : 0u;
                if (sp[j]) rw[j] = g.rankw[qv.push_w[u] + (v >> 6)];
            }
            uint32_t cnt = 0, tot = 0;
#pragma unroll
            for (int j = 0; j < SYM_BATCH; j++) {
                len[j] = 0;
                uint32_t e;
                if (sp[j] && row_range(g, rw[j], qv.push_r[u0 + j], v, beg[j], e)) {
                    if (e > beg[j] && e <= g.ncol) len[j] = e - beg[j];
                    else if (e != beg[j]) sviol(p);
                }
                if (len[j]) {
                    cnt++;
                    tot += len[j];
                }
            }
            uint64_t wtot;
            const uint64_t ex = wave_excl_scan((static_cast<uint64_t>(cnt) << 32) | tot, wtot);
            if (wtot == 0) continue;
            uint64_t old = 0;
            if (lane == 63)
                old = atomicAdd(reinterpret_cast<unsigned long long *>(&R.sel), static_cast<unsigned long long>(wtot));
            old = __shfl(old, 63, 64);
            if (cnt) {
                const uint64_t mine = old + ex;
                uint32_t idx = static_cast<uint32_t>(mine >> 32);
                uint32_t eb = static_cast<uint32_t>(mine);
#pragma unroll
                for (int j = 0; j < SYM_BATCH; j++) {
                    if (!len[j]) continue;
                    if (idx < p.item_cap) {
                        p.it_ebase[idx] = eb;
                        p.it_beg[idx] = beg[j];
                        p.it_v[idx] = v;
                        p.it_u[idx] = u0 + j;
                    } else {
                        sviol(p);
                    }
                    const uint32_t k1 = (eb + len[j] - 1) / TE;
                    for (uint32_t k = (eb + TE - 1) / TE; k <= k1; k++) {
                        if (k < p.tile_cap) p.tile_first[k] = idx;
                        else { sviol(p); break; }
                    }
                    idx++;
                    eb += len[j];
                }
            }
        }
    }
}

template <int G>
__device__ void st_push(const StackParams &p, uint32_t n, uint32_t *s_eb, uint32_t *s_beg, uint32_t *s_v,
                        uint32_t *s_u) {
    LevelRec *rec = p.rec;
    const uint64_t sel = ld_acq(&rec[n % REC_RING].sel);
    const uint32_t nitems = static_cast<uint32_t>(sel >> 32);
    const uint32_t T = static_cast<uint32_t>(sel);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.cnt[0] += nitems;
        p.cnt[1] += T;
        p.cnt[3] += ld_acq(&rec[n % REC_RING].nq);
    }
    if (T == 0 || nitems == 0) return;
    constexpr uint32_t TE = TILE / G;
    const uint32_t ntiles = (T + TE - 1) / TE;
    const uint32_t V = static_cast<uint32_t>(p.V);
    const QueryView &qv = p.qv;
    const uint64_t *Mc = p.M[n & 1];
    uint64_t *Mn = p.M[(n + 1) & 1];
    const uint32_t *sc = p.sup[n & 1];
    uint32_t *sn = p.sup[(n + 1) & 1];
    int32_t *qn = p.q[(n + 1) & 1];
    LevelRec &RN = rec[(n + 1) % REC_RING];
    const uint32_t tid = threadIdx.x;
    uint64_t pairs = 0, updates = 0;
    uint32_t su = 0;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        uint32_t i0 = tile < p.tile_cap ? p.tile_first[tile] : 0u;
        uint32_t i1 = (tile + 1 < ntiles && tile + 1 < p.tile_cap) ? p.tile_first[tile + 1] : nitems - 1;
        if (i0 >= nitems || i1 >= nitems || i1 < i0 || i1 - i0 > TE) {
            if (tid == 0) sviol(p);
            i0 = i1 = 0;
        }
        const uint32_t cnt = i1 - i0 + 1;
        for (uint32_t j = tid; j < cnt; j += BLOCK) {
            s_eb[j] = p.it_ebase[i0 + j];
            s_beg[j] = p.it_beg[i0 + j];
            s_v[j] = p.it_v[i0 + j];
            s_u[j] = p.it_u[i0 + j];
        }
        __syncthreads();
        const uint32_t t0 = tile * TE;
#pragma unroll
        for (int k = 0; k < TILE / BLOCK; k++) {
            const uint32_t unit = k * BLOCK + tid;
            const uint32_t t = t0 + unit / G;
            const uint32_t j = unit % G;
            uint32_t w = V, sbits = 0;
            if (t < T) {
                uint32_t lo = 0, hi = cnt;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s_eb[mid] <= t) lo = mid;
                    else hi = mid;
                }
                const uint32_t pos = s_beg[lo] + (t - s_eb[lo]);
                const uint32_t v = s_v[lo], u = s_u[lo];
                if (pos < p.g.ncol && v < V && u < qv.h->nsym) {
                    w = p.g.col[pos];
                    if (w >= V) sviol(p);
                } else {
                    sviol(p);
                }
                if (w < V) {
                    const uint32_t *succ = qv.succ + u * MAX_STATES;
                    uint32_t S = sc[v];
                    while (S) {
                        const uint32_t q = __ffs(S) - 1;
                        S &= S - 1;
                        uint32_t tq = succ[q];
                        if (!tq) continue;
                        const uint64_t x = Mc[row_index<G>(p, v, q) + j];
                        if (!x) continue;
                        while (tq) {
                            const uint32_t q2 = __ffs(tq) - 1;
                            tq &= tq - 1;
                            updates++;
                            const uint64_t idx = row_index<G>(p, w, q2) + j;
                            const uint64_t cand = x & ~p.P[idx];
                            if (!cand) continue;
                            const uint64_t nb =
                                cand & ~atomicOr(reinterpret_cast<unsigned long long *>(p.P + idx),
                                                 static_cast<unsigned long long>(cand));
                            if (!nb) continue;
                            atomicOr(reinterpret_cast<unsigned long long *>(Mn + idx), static_cast<unsigned long long>(nb));
                            sbits |= 1u << q2;
                            pairs += __popcll(nb);
                        }
                    }
                }
            }
            bool first = false;
            if (sbits) first = atomicOr(&sn[w], sbits) == 0;
            if (!wave_append(first, static_cast<int32_t>(w), qn, &RN.nq, V)) sviol(p);
            su |= sbits;
        }
        __syncthreads();
    }
    pairs = wave_sum(pairs);
    updates = wave_sum(updates);
    su = wave_or(su);
    if (lane_id() == 0 && pairs) {
        atomicAdd(reinterpret_cast<unsigned long long *>(&RN.pairs), (unsigned long long)pairs);
        atomicOr(&RN.su, su);
    }
    if (lane_id() == 0 && updates)
        atomicAdd(reinterpret_cast<unsigned long long *>(&p.cnt[2]), (unsigned long long)updates);
}

// Result: source b reaches v iff some final state's row at v has bit b. One
// wavefront per (64-vertex block, word): 64 ballots transpose the block into
// one output word per source. P and the last frontier are reset.
template <int G>
__device__ void st_final(const StackParams &p, uint32_t nlev) {
    const uint32_t V = static_cast<uint32_t>(p.V);
    const uint32_t Q = static_cast<uint32_t>(p.Q);
    if (nlev >= 1) {
        const uint32_t D = nlev - 1;
        const uint32_t nq = ld_acq(&p.rec[D % REC_RING].nq);
        uint64_t *M = p.M[D & 1];
        uint32_t *sp = p.sup[D & 1];
        const int32_t *q = p.q[D & 1];
        const uint64_t words = static_cast<uint64_t>(Q) * G;
        const uint64_t total = static_cast<uint64_t>(nq) * words;
        for (uint64_t x = gthread(); x < total; x += gthreads()) {
            const uint32_t v = static_cast<uint32_t>(q[x / words]);
            const uint32_t k = static_cast<uint32_t>(x % words);
            if (v >= V) {
                sviol(p);
                continue;
            }
            M[static_cast<uint64_t>(v) * words + k] = 0;
            if (k == 0) sp[v] = 0;
        }
    }
    const uint32_t fm = p.qv.h->fmask;
    const uint32_t lane = lane_id();
    const uint64_t nwords = static_cast<uint64_t>(p.nwords);
    const uint64_t total = nwords * G;
    const uint32_t B = static_cast<uint32_t>(p.B);
    for (uint64_t gw = gthread() >> 6; gw < total; gw += gthreads() >> 6) {
        const uint64_t k = gw / G;
        const uint32_t j = static_cast<uint32_t>(gw % G);
        const uint64_t v = k * 64 + lane;
        uint64_t f = 0;
        if (v < V) {
            for (uint32_t q = 0; q < Q; q++) {
                const uint64_t idx = row_index<G>(p, static_cast<uint32_t>(v), q) + j;
                const uint64_t x = p.P[idx];
                if (x) {
                    if (fm >> q & 1u) f |= x;
                    p.P[idx] = 0;
                }
            }
        }
        for (uint32_t i = 0; i < 64; i++) {
            const uint64_t b = __ballot((f >> i) & 1ull);
            const uint32_t src = j * 64 + i;
            if (lane == 0 && src < B) p.out[static_cast<uint64_t>(src) * nwords + k] = b;
        }
    }
}

template <int G>
__global__ __launch_bounds__(BLOCK) void k_stacked(StackParams p) {
    __shared__ uint32_t s_eb[TILE + 1], s_beg[TILE + 1], s_v[TILE + 1], s_u[TILE + 1];
    GridBarrier *bar = p.bar;
    BarCtx bc;
    if (!barrier_register(bar, bc)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.rec[0] = LevelRec{};
        for (int i = 0; i < 4; i++) p.status[i] = 0;
        for (int i = 0; i < 4; i++) p.cnt[i] = 0;
    }
    if (!grid_barrier(bar, bc)) return;
    // start pairs: every source's bit in every start state's row
    const QHeader &h = *p.qv.h;
    const uint32_t V = static_cast<uint32_t>(p.V);
    for (uint32_t i = gthread(); i < static_cast<uint32_t>(p.B); i += gthreads()) {
        const uint32_t s = static_cast<uint32_t>(p.sources[i]);
        if (s >= V || !h.smask) {
            if (s >= V) sviol(p);
            continue;
        }
        const uint64_t bit = 1ull << (i & 63);
        uint32_t sm = h.smask;
        while (sm) {
            const uint32_t q = __ffs(sm) - 1;
            sm &= sm - 1;
            const uint64_t idx = row_index<G>(p, s, q) + (i >> 6);
            atomicOr(reinterpret_cast<unsigned long long *>(p.P + idx), static_cast<unsigned long long>(bit));
            atomicOr(reinterpret_cast<unsigned long long *>(p.M[0] + idx), static_cast<unsigned long long>(bit));
        }
        if (atomicOr(&p.sup[0][s], h.smask) == 0) {
            const uint32_t pos = atomicAdd(&p.rec[0].nq, 1u);
            if (pos < V) p.q[0][pos] = static_cast<int32_t>(s);
            else sviol(p);
        }
        atomicAdd(reinterpret_cast<unsigned long long *>(&p.rec[0].pairs),
                  static_cast<unsigned long long>(__popc(h.smask)));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) p.rec[0].su = h.smask;
    if (!grid_barrier(bar, bc)) return;
    uint32_t n = 0;
    while (true) {
        if (ld_acq(&p.rec[n % REC_RING].nq) == 0) break;
        st_select<G>(p, n);
        if (!grid_barrier(bar, bc)) return;
        st_push<G>(p, n, s_eb, s_beg, s_v, s_u);
        if (!grid_barrier(bar, bc)) return;
        n++;
    }
    st_final<G>(p, n);
    if (blockIdx.x == 0 && threadIdx.x == 0) p.status[0] = n;
}

template <int G>
static hipError_t launch_g(const StackParams &p, int grid, hipStream_t s) {
    StackParams a = p;
    void *args[] = {&a};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_stacked<G>), dim3(grid), dim3(BLOCK), args,
                                      0, s);
}

hipError_t launch_stacked(int G, const StackParams &p, int grid, hipStream_t s) {
    switch (G) {
        case 1: return launch_g<1>(p, grid, s);
        case 2: return launch_g<2>(p, grid, s);
        case 4: return launch_g<4>(p, grid, s);
        case 8: return launch_g<8>(p, grid, s);
        default: return launch_g<16>(p, grid, s);
    }
}

int stacked_grid(int G) {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e;
    switch (G) {
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_stacked<1>, BLOCK, 0); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_stacked<2>, BLOCK, 0); break;
        case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_stacked<4>, BLOCK, 0); break;
        case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_stacked<8>, BLOCK, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_stacked<16>, BLOCK, 0); break;
    }
    if (e != hipSuccess || per < 1) return 0;
    return ncu * (per < PERSISTENT_BLOCKS_PER_CU ? per : PERSISTENT_BLOCKS_PER_CU);
}

}  // namespace rpq
