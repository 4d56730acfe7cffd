// HIP kernels for one single-source query on gfx950 (64-lane wavefronts).
//
// One level of Alg. 1 (Sec. 4) computes
//     M' = ( sum_a (N^a)^T M G^a ) masked by not-P,      P = P + M'
// over the Boolean semiring. The kernels never form a matrix. Per vertex the
// |Q| states of M and P are one bit-packed word (1, 2 or 4 bytes), and a level
// runs as three phases:
//
//  select  for every frontier vertex v and every segment (v, label) of the
//          symbols the query uses, the product (N^a)^T M restricted to column v
//          is the successor set succ_a(M[v]) (a few table ORs); each non-empty
//          one becomes a push item (neighbour range, state set). This applies
//          the small NFA factor first, the evaluation order Sec. 4 recommends.
//  push    the items' edges are spread evenly over the grid; each edge (v, w)
//          ORs the item's set into P[w] with one atomic; the bits that were
//          not yet set (the not-P mask) go to M'[w], and the first writer of
//          M'[w] appends w to the next frontier queue (wave ballot + popc).
//  pull    used instead of push on dense levels: every vertex w with states
//          still unvisited scans its reverse neighbours under the symbols that
//          can reach those states and stops as soon as all are found.
//
// Inverse symbols a^- read the transposed adjacency (Sec. 3: G^{a^-} = (G^a)^T):
// the graph store holds both directions, and the label -> symbol tables map an
// IN segment to the inverse symbol of its label.
//
// The whole traversal runs as one cooperative launch with grid barriers
// between phases (no host round trip per level); the same phase code is also
// launched kernel by kernel for the host-driven loop.
#include <hip/hip_runtime.h>

#include "rpq_internal.h"

namespace rpq {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

template <int W>
__device__ __forceinline__ uint32_t ld_state(const uint32_t *a, uint32_t v) {
    if constexpr (W == 4) return a[v];
    else if constexpr (W == 2) return reinterpret_cast<const uint16_t *>(a)[v];
    else return reinterpret_cast<const uint8_t *>(a)[v];
}

template <int W>
__device__ __forceinline__ void st_state(uint32_t *a, uint32_t v, uint32_t x) {
    if constexpr (W == 4) a[v] = x;
    else if constexpr (W == 2) reinterpret_cast<uint16_t *>(a)[v] = static_cast<uint16_t>(x);
    else reinterpret_cast<uint8_t *>(a)[v] = static_cast<uint8_t>(x);
}

// Atomic OR of x into vertex v's sub-word; returns the sub-word's old value.
template <int W>
__device__ __forceinline__ uint32_t or_state(uint32_t *a, uint32_t v, uint32_t x) {
    if constexpr (W == 4) {
        return atomicOr(a + v, x);
    } else {
        constexpr uint32_t per = 4 / W;
        constexpr uint32_t mask = (1u << (8 * W)) - 1u;
        const uint32_t sh = (v % per) * (8 * W);
        return (atomicOr(a + v / per, x << sh) >> sh) & mask;
    }
}

template <typename T>
__device__ __forceinline__ T ld_acq(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t wave_excl_scan(uint64_t x, uint64_t &total) {
    const uint32_t lane = lane_id();
    uint64_t inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(inc, d, 64);
        if (lane >= static_cast<uint32_t>(d)) inc += y;
    }
    total = __shfl(inc, 63, 64);
    return inc - x;
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x |= __shfl_xor(x, d, 64);
    return x;
}

// Appends `value` for every lane with `flag` to queue[*counter ...] with one
// atomic per wave. All 64 lanes must call it.
__device__ __forceinline__ void wave_append(bool flag, int32_t value, int32_t *queue,
                                            uint32_t *counter) {
    const uint64_t m = __ballot(flag);
    if (m == 0) return;
    const uint32_t lane = lane_id();
    const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
    uint32_t base = 0;
    if (static_cast<int>(lane) == leader) base = atomicAdd(counter, static_cast<uint32_t>(__popcll(m)));
    base = __shfl(base, leader, 64);
    if (flag) queue[base + __popcll(m & ((1ull << lane) - 1ull))] = value;
}

__device__ __forceinline__ uint32_t succ_of(const uint32_t *succ, uint32_t u, uint32_t S) {
    const uint32_t *t = succ + u * MAX_STATES;
    uint32_t r = 0;
    while (S) {
        r |= t[__ffs(S) - 1];
        S &= S - 1;
    }
    return r;
}

__device__ __forceinline__ uint32_t count_succ(const uint32_t *succ, uint32_t u, uint32_t S) {
    const uint32_t *t = succ + u * MAX_STATES;
    uint32_t c = 0;
    while (S) {
        c += __popc(t[__ffs(S) - 1]);
        S &= S - 1;
    }
    return c;
}

__device__ __forceinline__ uint32_t gthread() { return blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ uint32_t gthreads() { return gridDim.x * blockDim.x; }

// Grid-wide barrier for the persistent kernel (all workgroups co-resident, as
// the cooperative launch guarantees). Each XCD has its own L2, so arrival is a
// device-scope release (dirty lines written back) and departure a
// device-scope acquire (stale lines dropped). The wait is bounded in time:
// after BARRIER_TIMEOUT ticks of the 100 MHz wall clock the barrier records an
// abort and every workgroup leaves the kernel at its next barrier.
constexpr uint64_t BARRIER_TIMEOUT = 5ull * 100000000ull;  // 5 s

__device__ bool grid_barrier(GridBarrier *b) {
    __syncthreads();
    __shared__ uint32_t s_ok;
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t gen = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t arrived =
            __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t ok = 1;
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&b->gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(&b->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                if (wall_clock64() - t0 > BARRIER_TIMEOUT) {
                    __hip_atomic_store(&b->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (__hip_atomic_load(&b->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// ---------------------------------------------------------------- phases
template <int W>
__device__ void init_phase(const Params &p) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const QHeader &h = *p.qv.h;
    LevelRec *r = p.st.rec;
    r[0] = LevelRec{};
    const uint32_t sm = h.smask;
    if (sm) {
        st_state<W>(p.st.P, p.source, sm);
        st_state<W>(p.st.M[0], p.source, sm);
        p.st.q[0][0] = p.source;
        r[0].nq = 1;
        r[0].su = sm;
        r[0].pairs = __popc(sm);
    }
    for (int i = 0; i < 4; i++) p.st.cnt[i] = 0;
    p.st.status[0] = p.st.status[1] = p.st.status[2] = 0;
}

template <int W>
__device__ void select_phase(const Params &p, uint32_t n) {
    const GraphView &g = p.g;
    const QHeader &h = *p.qv.h;
    LevelRec *rec = p.st.rec;
    LevelRec &R = rec[n % REC_RING];
    const uint32_t nq = ld_acq(&R.nq);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rec[(n + 1) % REC_RING] = LevelRec{};
        if (n < LVL_COUNT_CAP) p.st.lvl_pairs[n] = static_cast<int64_t>(ld_acq(&R.pairs));
        if (h.counters) p.st.cnt[3] += nq;
    }
    // frontier words of level n-1 live in the buffer level n writes: clear them
    if (n >= 1) {
        const uint32_t nprev = ld_acq(&rec[(n - 1) % REC_RING].nq);
        uint32_t *Mold = p.st.M[(n + 1) & 1];
        const int32_t *qold = p.st.q[(n + 1) & 1];
        for (uint32_t i = gthread(); i < nprev; i += gthreads()) st_state<W>(Mold, qold[i], 0);
    }
    const int32_t *qc = p.st.q[n & 1];
    const uint32_t *Mc = p.st.M[n & 1];
    const uint32_t lane = lane_id();
    const uint32_t gw = gthread() >> 6, nw = gthreads() >> 6;
    uint64_t c_pe = 0, c_sc = 0, c_sd = 0;
    for (uint32_t base = gw * 64; base < nq; base += nw * 64) {
        const uint32_t i = base + lane;
        const bool act = i < nq;
        const uint32_t v = act ? static_cast<uint32_t>(qc[i]) : 0u;
        const uint32_t S = act ? ld_state<W>(Mc, v) : 0u;
        uint32_t cnt = 0, len = 0;
        if (S) {
            for (int d = 0; d < 2; d++) {
                const uint32_t s0 = g.vseg[d][v], s1 = g.vseg[d][v + 1];
                for (uint32_t s = s0; s < s1; s++) {
                    const int u = p.qv.l2s[d][g.seg_lab[d][s]];
                    if (u < 0) continue;
                    const uint32_t ln = g.seg_beg[d][s + 1] - g.seg_beg[d][s];
                    if (ln == 0) continue;
                    if (h.counters) c_pe += static_cast<uint64_t>(count_succ(p.qv.succ, u, S)) * ln;
                    if (!succ_of(p.qv.succ, u, S)) continue;
                    cnt++;
                    len += ln;
                }
            }
        }
        if (h.counters) {
            c_sc += cnt;
            c_sd += len;
        }
        uint64_t tot;
        const uint64_t ex = wave_excl_scan((static_cast<uint64_t>(cnt) << 32) | len, tot);
        if (tot == 0) continue;
        uint64_t old = 0;
        if (lane == 63) old = atomicAdd(reinterpret_cast<unsigned long long *>(&R.sel),
                                        static_cast<unsigned long long>(tot));
        old = __shfl(old, 63, 64);
        if (cnt) {
            const uint64_t mine = old + ex;
            uint32_t idx = static_cast<uint32_t>(mine >> 32);
            uint32_t eb = static_cast<uint32_t>(mine);
            for (int d = 0; d < 2; d++) {
                const uint32_t s0 = g.vseg[d][v], s1 = g.vseg[d][v + 1];
                for (uint32_t s = s0; s < s1; s++) {
                    const int u = p.qv.l2s[d][g.seg_lab[d][s]];
                    if (u < 0) continue;
                    const uint32_t sp = succ_of(p.qv.succ, u, S);
                    if (!sp) continue;
                    const uint32_t b = g.seg_beg[d][s];
                    const uint32_t ln = g.seg_beg[d][s + 1] - b;
                    if (ln == 0) continue;  // never built; keeps the tile loop bounded
                    p.st.it_ebase[idx] = eb;
                    p.st.it_beg[idx] = b;
                    p.st.it_mask[idx] = sp;
                    // this item owns the tiles whose first edge falls inside it
                    for (uint32_t k = (eb + TILE - 1) / TILE; k <= (eb + ln - 1) / TILE; k++)
                        p.st.tile_first[k] = idx;
                    idx++;
                    eb += ln;
                }
            }
        }
    }
    if (h.counters) {
        c_pe = wave_sum(c_pe);
        c_sc = wave_sum(c_sc);
        c_sd = wave_sum(c_sd);
        if (lane == 0 && (c_pe | c_sc)) {
            atomicAdd(reinterpret_cast<unsigned long long *>(&p.st.cnt[0]), (unsigned long long)c_pe);
            atomicAdd(reinterpret_cast<unsigned long long *>(&p.st.cnt[1]), (unsigned long long)c_sc);
            atomicAdd(reinterpret_cast<unsigned long long *>(&p.st.cnt[2]), (unsigned long long)c_sd);
        }
    }
}

// push (0) or pull (1) for level n; every workgroup computes the same answer
__device__ __forceinline__ uint32_t decide(const Params &p, uint32_t n) {
    const QHeader &h = *p.qv.h;
    if (h.force == 1) return 0;
    if (h.force == 2) return 1;
    if (!(h.alpha > 0.f)) return 0;
    const LevelRec *rec = p.st.rec;
    const uint32_t prev = n ? ld_acq(&rec[(n - 1) % REC_RING].mode) : 0u;
    const uint64_t T = ld_acq(&rec[n % REC_RING].sel) & 0xffffffffull;
    const uint32_t nq = ld_acq(&rec[n % REC_RING].nq);
    if (prev == 0) return static_cast<double>(T) * h.alpha > static_cast<double>(h.e_rel) ? 1u : 0u;
    return static_cast<double>(nq) * h.beta < static_cast<double>(p.g.V) ? 0u : 1u;
}

template <int W>
__device__ void push_phase(const Params &p, uint32_t n, uint32_t *s_eb, uint32_t *s_beg,
                           uint32_t *s_mask) {
    LevelRec *rec = p.st.rec;
    const uint64_t sel = ld_acq(&rec[n % REC_RING].sel);
    const uint32_t nitems = static_cast<uint32_t>(sel >> 32);
    const uint32_t T = static_cast<uint32_t>(sel);
    if (T == 0) return;
    const uint32_t ntiles = (T + TILE - 1) / TILE;
    uint32_t *P = p.st.P;
    uint32_t *Mn = p.st.M[(n + 1) & 1];
    int32_t *qn = p.st.q[(n + 1) & 1];
    LevelRec &RN = rec[(n + 1) % REC_RING];
    const uint32_t *col = p.g.col;
    const uint32_t tid = threadIdx.x;
    uint64_t pairs = 0;
    uint32_t su = 0;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t i0 = p.st.tile_first[tile];
        const uint32_t i1 = tile + 1 < ntiles ? p.st.tile_first[tile + 1] : nitems - 1;
        const uint32_t cnt = i1 - i0 + 1;  // <= TILE + 1
        for (uint32_t j = tid; j < cnt; j += BLOCK) {
            s_eb[j] = p.st.it_ebase[i0 + j];
            s_beg[j] = p.st.it_beg[i0 + j];
            s_mask[j] = p.st.it_mask[i0 + j];
        }
        __syncthreads();
        const uint32_t t0 = tile * TILE;
#pragma unroll
        for (int k = 0; k < TILE / BLOCK; k++) {
            const uint32_t t = t0 + k * BLOCK + tid;
            bool first = false;
            uint32_t w = 0, nwd = 0;
            if (t < T) {
                uint32_t lo = 0, hi = cnt;  // s_eb[lo] <= t < s_eb[hi]
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s_eb[mid] <= t) lo = mid;
                    else hi = mid;
                }
                w = col[s_beg[lo] + (t - s_eb[lo])];
                const uint32_t sp = s_mask[lo];
                const uint32_t cand = sp & ~ld_state<W>(P, w);
                if (cand) {
                    nwd = cand & ~or_state<W>(P, w, cand);
                    if (nwd) first = or_state<W>(Mn, w, nwd) == 0;
                }
            }
            wave_append(first, static_cast<int32_t>(w), qn, &RN.nq);
            pairs += __popc(nwd);
            su |= nwd;
        }
        __syncthreads();
    }
    pairs = wave_sum(pairs);
    su = wave_or(su);
    if (lane_id() == 0 && pairs) {
        atomicAdd(reinterpret_cast<unsigned long long *>(&RN.pairs), (unsigned long long)pairs);
        atomicOr(&RN.su, su);
    }
}

template <int W>
__device__ void pull_phase(const Params &p, uint32_t n) {
    const GraphView &g = p.g;
    const QHeader &h = *p.qv.h;
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
    uint32_t *P = p.st.P;
    LevelRec &RN = rec[(n + 1) % REC_RING];
    const uint32_t lane = lane_id();
    const uint32_t gw = gthread() >> 6, nw = gthreads() >> 6;
    const uint32_t V = static_cast<uint32_t>(g.V);
    uint64_t pairs = 0;
    uint32_t sacc = 0;
    for (uint32_t base = gw * 64; base < V; base += nw * 64) {
        const uint32_t w = base + lane;
        uint32_t acc = 0;
        if (w < V) {
            const uint32_t pw = ld_state<W>(P, w);
            const uint32_t U = ns & ~pw;
            if (U) {
                // IN segments of w carry forward symbols, OUT segments inverse ones
                for (int d = 1; d >= 0 && acc != U; d--) {
                    const int16_t *l2s = p.qv.l2s[1 - d];
                    const uint32_t s0 = g.vseg[d][w], s1 = g.vseg[d][w + 1];
                    for (uint32_t s = s0; s < s1 && acc != U; s++) {
                        const int u = l2s[g.seg_lab[d][s]];
                        if (u < 0) continue;
                        uint32_t pu = succ_of(p.qv.pred, u, U & ~acc);
                        if (!pu) continue;
                        const uint32_t e1 = g.seg_beg[d][s + 1];
                        for (uint32_t e = g.seg_beg[d][s]; e < e1; e++) {
                            const uint32_t m = ld_state<W>(Mc, g.col[e]) & pu;
                            if (m) {
                                acc |= succ_of(p.qv.succ, u, m) & U;
                                if (acc == U) break;
                                pu = succ_of(p.qv.pred, u, U & ~acc);
                                if (!pu) break;
                            }
                        }
                    }
                }
                if (acc) {
                    st_state<W>(P, w, pw | acc);
                    st_state<W>(Mn, w, acc);
                }
            }
        }
        wave_append(acc != 0, static_cast<int32_t>(w), qn, &RN.nq);
        pairs += __popc(acc);
        sacc |= acc;
    }
    pairs = wave_sum(pairs);
    sacc = wave_or(sacc);
    if (lane == 0 && pairs) {
        atomicAdd(reinterpret_cast<unsigned long long *>(&RN.pairs), (unsigned long long)pairs);
        atomicOr(&RN.su, sacc);
    }
}

// Clears the last frontier's words, writes the result bitmap (vertex v has a
// final state: the product F P of Alg. 1) and resets P for the next query.
template <int W>
__device__ void final_phase(const Params &p, uint32_t nlev) {
    if (nlev >= 1) {
        const uint32_t D = nlev - 1;
        const uint32_t nq = ld_acq(&p.st.rec[D % REC_RING].nq);
        uint32_t *M = p.st.M[D & 1];
        const int32_t *q = p.st.q[D & 1];
        for (uint32_t i = gthread(); i < nq; i += gthreads()) st_state<W>(M, q[i], 0);
    }
    const uint32_t fm = p.qv.h->fmask;
    const uint32_t V = static_cast<uint32_t>(p.g.V);
    const uint32_t nwords = (V + 63) / 64;
    const uint32_t lane = lane_id();
    const uint32_t gw = gthread() >> 6, nw = gthreads() >> 6;
    for (uint32_t k = gw; k < nwords; k += nw) {
        const uint32_t v = k * 64 + lane;
        const uint32_t pv = v < V ? ld_state<W>(p.st.P, v) : 0u;
        const uint64_t b = __ballot((pv & fm) != 0);
        if (lane == 0) p.st.out[k] = b;
        if (pv) st_state<W>(p.st.P, v, 0);
    }
}

// ---------------------------------------------------------------- kernels
template <int W>
__global__ __launch_bounds__(BLOCK) void k_persistent(Params p) {
    __shared__ uint32_t s_eb[TILE + 1], s_beg[TILE + 1], s_mask[TILE + 1];
    GridBarrier *bar = p.st.bar;
    init_phase<W>(p);
    if (!grid_barrier(bar)) return;
    uint32_t n = 0, npush = 0, npull = 0;
    while (true) {
        if (ld_acq(&p.st.rec[n % REC_RING].nq) == 0) break;
        select_phase<W>(p, n);
        if (!grid_barrier(bar)) return;
        const uint32_t mode = decide(p, n);
        if (blockIdx.x == 0 && threadIdx.x == 0) p.st.rec[n % REC_RING].mode = mode;
        if (mode == 0) push_phase<W>(p, n, s_eb, s_beg, s_mask);
        else pull_phase<W>(p, n);
        npush += mode == 0;
        npull += mode != 0;
        if (!grid_barrier(bar)) return;
        n++;
    }
    final_phase<W>(p, n);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.st.status[0] = n;
        p.st.status[1] = npush;
        p.st.status[2] = npull;
    }
}

template <int W>
__global__ __launch_bounds__(64) void k_init(Params p) {
    init_phase<W>(p);
}

template <int W>
__global__ __launch_bounds__(BLOCK) void k_select(Params p, uint32_t n) {
    select_phase<W>(p, n);
}

template <int W>
__global__ __launch_bounds__(BLOCK) void k_expand(Params p, uint32_t n) {
    __shared__ uint32_t s_eb[TILE + 1], s_beg[TILE + 1], s_mask[TILE + 1];
    const uint32_t mode = decide(p, n);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.st.rec[n % REC_RING].mode = mode;
        p.st.status[0] = n + 1;
        p.st.status[1 + (mode != 0)] += 1;
    }
    if (mode == 0) push_phase<W>(p, n, s_eb, s_beg, s_mask);
    else pull_phase<W>(p, n);
}

template <int W>
__global__ __launch_bounds__(BLOCK) void k_final(Params p, uint32_t nlev) {
    final_phase<W>(p, nlev);
}

__global__ void k_fill(uint32_t *ptr, uint64_t words, uint32_t value) {
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        ptr[i] = value;
}

// ---------------------------------------------------------------- launchers
template <int W>
static hipError_t launch_persistent_w(const Params &p, int grid, hipStream_t s) {
    Params a = p;
    void *args[] = {&a};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_persistent<W>), dim3(grid),
                                      dim3(BLOCK), args, 0, s);
}

hipError_t launch_persistent(int W, const Params &p, int grid, hipStream_t s) {
    switch (W) {
        case 1: return launch_persistent_w<1>(p, grid, s);
        case 2: return launch_persistent_w<2>(p, grid, s);
        default: return launch_persistent_w<4>(p, grid, s);
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
