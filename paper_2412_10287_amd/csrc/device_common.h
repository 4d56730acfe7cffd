// Device helpers shared by the single-query and multi-query kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "rpq_internal.h"

namespace rpq {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// State word of vertex v (a device-scope load: see ldc).
template <int W>
__device__ __forceinline__ uint32_t ld_state(const uint32_t *a, uint32_t v) {
    if constexpr (W == 4) return __hip_atomic_load(a + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else if constexpr (W == 2)
        return __hip_atomic_load(reinterpret_cast<const uint16_t *>(a) + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return __hip_atomic_load(reinterpret_cast<const uint8_t *>(a) + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Load of data that other workgroups write during a persistent launch
// (queues, state words, items): a device-scope load, which misses the
// compute unit's L1. The grid barrier invalidates the L1 only in the XCD
// leaders (the invalidations of all workgroups queue up in each XCD), so
// every such read in the persistent kernels goes through here.
template <typename T>
__device__ __forceinline__ T ldc(const T *p) {
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
// atomic per wave. All 64 lanes must call it. Returns false if this lane's
// slot would be at or beyond `cap` (then nothing is written).
__device__ __forceinline__ bool wave_append(bool flag, int32_t value, int32_t *queue, uint32_t *counter,
                                            uint32_t cap) {
    const uint64_t m = __ballot(flag);
    if (m == 0) return true;
    const uint32_t lane = lane_id();
    const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
    uint32_t base = 0;
    if (static_cast<int>(lane) == leader) base = atomicAdd(counter, static_cast<uint32_t>(__popcll(m)));
    base = __shfl(base, leader, 64);
    if (!flag) return true;
    const uint32_t pos = base + static_cast<uint32_t>(__popcll(m & ((1ull << lane) - 1ull)));
    if (pos >= cap) return false;
    queue[pos] = value;
    return true;
}

// wave_append for four (flag, value) pairs per lane with one atomic per wave.
__device__ __forceinline__ bool wave_append4(bool f0, int32_t v0, bool f1, int32_t v1, bool f2, int32_t v2, bool f3,
                                             int32_t v3, int32_t *queue, uint32_t *counter, uint32_t cap) {
    const uint64_t m0 = __ballot(f0), m1 = __ballot(f1), m2 = __ballot(f2), m3 = __ballot(f3);
    const uint32_t c0 = static_cast<uint32_t>(__popcll(m0)), c1 = static_cast<uint32_t>(__popcll(m1));
    const uint32_t c2 = static_cast<uint32_t>(__popcll(m2)), c3 = static_cast<uint32_t>(__popcll(m3));
    const uint32_t tot = c0 + c1 + c2 + c3;
    if (tot == 0) return true;
    const uint32_t lane = lane_id();
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(counter, tot);
    base = __shfl(base, 0, 64);
    const uint64_t below = (1ull << lane) - 1ull;
    bool ok = true;
    uint32_t pos;
    if (f0) {
        pos = base + static_cast<uint32_t>(__popcll(m0 & below));
        if (pos < cap) queue[pos] = v0;
        else ok = false;
    }
    if (f1) {
        pos = base + c0 + static_cast<uint32_t>(__popcll(m1 & below));
        if (pos < cap) queue[pos] = v1;
        else ok = false;
    }
    if (f2) {
        pos = base + c0 + c1 + static_cast<uint32_t>(__popcll(m2 & below));
        if (pos < cap) queue[pos] = v2;
        else ok = false;
    }
    if (f3) {
        pos = base + c0 + c1 + c2 + static_cast<uint32_t>(__popcll(m3 & below));
        if (pos < cap) queue[pos] = v3;
        else ok = false;
    }
    return ok;
}

// ------------------------------------------------- workgroup aggregation
// Atomics on one address are serialised (about 12 ns each on MI355X), so a
// counter that every wave of the grid updates once per step is a bottleneck
// at a few thousand waves. The helpers below let a workgroup make one atomic
// where its waves would make eight. Every thread of the workgroup must call
// them (workgroup-uniform control flow; blockDim.x == BLOCK).
constexpr int NWAVE = BLOCK / 64;

__device__ __forceinline__ uint32_t atomic_add_any(uint32_t *p, uint32_t x) { return atomicAdd(p, x); }
__device__ __forceinline__ uint64_t atomic_add_any(uint64_t *p, uint64_t x) {
    return atomicAdd(reinterpret_cast<unsigned long long *>(p), static_cast<unsigned long long>(x));
}

// Reserves the workgroup's summed amount on `counter` with one atomic; `wtot`
// is the calling wave's amount (the same in all its lanes). base receives the
// wave's first position (its share follows the shares of the lower waves).
// Also returns whether any lane of the workgroup passed more == true.
template <typename T>
__device__ __forceinline__ bool block_reserve(T wtot, bool more, T *counter, T &base) {
    __shared__ T s_w[NWAVE];
    __shared__ uint32_t s_more[NWAVE];
    __shared__ T s_base;
    const uint32_t wave = threadIdx.x >> 6;
    const bool wmore = __ballot(more) != 0;
    if (lane_id() == 0) {
        s_w[wave] = wtot;
        s_more[wave] = wmore ? 1u : 0u;
    }
    __syncthreads();
    T off = 0, tot = 0;
    uint32_t any = 0;
#pragma unroll
    for (int k = 0; k < NWAVE; k++) {
        const T x = s_w[k];
        if (static_cast<uint32_t>(k) < wave) off += x;
        tot += x;
        any |= s_more[k];
    }
    if (threadIdx.x == 0 && tot) s_base = atomic_add_any(counter, tot);
    __syncthreads();
    base = tot ? s_base + off : T(0);
    return any != 0;
}

// block_reserve on two counters at once (same synchronisation cost as one):
// a 64-bit amount w64 on c64 and a 32-bit amount w32 on c32.
__device__ __forceinline__ void block_reserve2(uint64_t w64, uint64_t *c64, uint64_t &b64, uint32_t w32,
                                               uint32_t *c32, uint32_t &b32) {
    __shared__ uint64_t s_w64[NWAVE], s_b64;
    __shared__ uint32_t s_w32[NWAVE], s_b32;
    const uint32_t wave = threadIdx.x >> 6;
    if (lane_id() == 0) {
        s_w64[wave] = w64;
        s_w32[wave] = w32;
    }
    __syncthreads();
    uint64_t off64 = 0, tot64 = 0;
    uint32_t off32 = 0, tot32 = 0;
#pragma unroll
    for (int k = 0; k < NWAVE; k++) {
        const uint64_t x = s_w64[k];
        const uint32_t y = s_w32[k];
        if (static_cast<uint32_t>(k) < wave) {
            off64 += x;
            off32 += y;
        }
        tot64 += x;
        tot32 += y;
    }
    if (threadIdx.x == 0 && tot64) s_b64 = atomic_add_any(c64, tot64);
    if (threadIdx.x == 64 && tot32) s_b32 = atomic_add_any(c32, tot32);
    __syncthreads();
    b64 = tot64 ? s_b64 + off64 : 0ull;
    b32 = tot32 ? s_b32 + off32 : 0u;
}

// wave_append4 with one queue reservation per workgroup and step.
__device__ __forceinline__ bool block_append4(bool f0, int32_t v0, bool f1, int32_t v1, bool f2, int32_t v2, bool f3,
                                              int32_t v3, int32_t *queue, uint32_t *counter, uint32_t cap) {
    const uint64_t m0 = __ballot(f0), m1 = __ballot(f1), m2 = __ballot(f2), m3 = __ballot(f3);
    const uint32_t c0 = static_cast<uint32_t>(__popcll(m0)), c1 = static_cast<uint32_t>(__popcll(m1));
    const uint32_t c2 = static_cast<uint32_t>(__popcll(m2)), c3 = static_cast<uint32_t>(__popcll(m3));
    const uint32_t tot = c0 + c1 + c2 + c3;
    uint32_t base = 0;
    block_reserve<uint32_t>(tot, false, counter, base);
    if (tot == 0) return true;
    const uint64_t below = (1ull << lane_id()) - 1ull;
    bool ok = true;
    uint32_t pos;
    if (f0) {
        pos = base + static_cast<uint32_t>(__popcll(m0 & below));
        if (pos < cap) queue[pos] = v0;
        else ok = false;
    }
    if (f1) {
        pos = base + c0 + static_cast<uint32_t>(__popcll(m1 & below));
        if (pos < cap) queue[pos] = v1;
        else ok = false;
    }
    if (f2) {
        pos = base + c0 + c1 + static_cast<uint32_t>(__popcll(m2 & below));
        if (pos < cap) queue[pos] = v2;
        else ok = false;
    }
    if (f3) {
        pos = base + c0 + c1 + c2 + static_cast<uint32_t>(__popcll(m3 & below));
        if (pos < cap) queue[pos] = v3;
        else ok = false;
    }
    return ok;
}

// wave_append with one queue reservation per workgroup.
__device__ __forceinline__ bool block_append(bool flag, int32_t value, int32_t *queue, uint32_t *counter,
                                             uint32_t cap) {
    const uint64_t m = __ballot(flag);
    uint32_t base = 0;
    block_reserve<uint32_t>(static_cast<uint32_t>(__popcll(m)), false, counter, base);
    if (!flag) return true;
    const uint32_t pos = base + static_cast<uint32_t>(__popcll(m & ((1ull << lane_id()) - 1ull)));
    if (pos >= cap) return false;
    queue[pos] = value;
    return true;
}

// block_reserve for a cursor that one workgroup alone advances: `running`
// (the same in every thread) takes the place of the counter in memory, so no
// atomic is made. base receives the wave's first position.
template <typename T>
__device__ __forceinline__ bool block_reserve_local(T wtot, bool more, T &running, T &base) {
    __shared__ T s_w[NWAVE];
    __shared__ uint32_t s_more[NWAVE];
    const uint32_t wave = threadIdx.x >> 6;
    const bool wmore = __ballot(more) != 0;
    if (lane_id() == 0) {
        s_w[wave] = wtot;
        s_more[wave] = wmore ? 1u : 0u;
    }
    __syncthreads();
    T off = 0, tot = 0;
    uint32_t any = 0;
#pragma unroll
    for (int k = 0; k < NWAVE; k++) {
        const T x = s_w[k];
        if (static_cast<uint32_t>(k) < wave) off += x;
        tot += x;
        any |= s_more[k];
    }
    __syncthreads();  // s_w is read everywhere before the next call writes it
    base = running + off;
    running += tot;
    return any != 0;
}

// block_append4 for a queue that one workgroup alone fills, kept twice: in
// `lq` (positions below lcap; the rest are dropped) and in `gq` (positions
// below gcap; returns false if this lane's slots go beyond). `running` is the
// queue length, the same in every thread.
__device__ __forceinline__ bool block_append4_local(bool f0, int32_t v0, bool f1, int32_t v1, bool f2, int32_t v2,
                                                    bool f3, int32_t v3, int32_t *lq, uint32_t lcap, int32_t *gq,
                                                    uint32_t gcap, uint32_t &running) {
    const uint64_t m0 = __ballot(f0), m1 = __ballot(f1), m2 = __ballot(f2), m3 = __ballot(f3);
    const uint32_t c0 = static_cast<uint32_t>(__popcll(m0)), c1 = static_cast<uint32_t>(__popcll(m1));
    const uint32_t c2 = static_cast<uint32_t>(__popcll(m2)), c3 = static_cast<uint32_t>(__popcll(m3));
    const uint32_t tot = c0 + c1 + c2 + c3;
    uint32_t base = 0;
    block_reserve_local<uint32_t>(tot, false, running, base);
    if (tot == 0) return true;
    const uint64_t below = (1ull << lane_id()) - 1ull;
    bool ok = true;
    const bool f[4] = {f0, f1, f2, f3};
    const int32_t v[4] = {v0, v1, v2, v3};
    const uint64_t m[4] = {m0, m1, m2, m3};
    uint32_t pre = base;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if (f[k]) {
            const uint32_t pos = pre + static_cast<uint32_t>(__popcll(m[k] & below));
            if (pos < lcap) lq[pos] = v[k];
            if (pos < gcap) gq[pos] = v[k];
            else ok = false;
        }
        pre += static_cast<uint32_t>(__popcll(m[k]));
    }
    return ok;
}

// Totals over the workgroup of K per-wave values (already reduced over the
// wave: the same in all its lanes): sums, or ORs for the k with bit k of
// or_mask set. Thread k < K receives total k, every other thread 0.
template <int K>
__device__ __forceinline__ uint64_t block_reduce(const uint64_t (&v)[K], uint32_t or_mask) {
    __shared__ uint64_t s_part[NWAVE][K];
    const uint32_t wave = threadIdx.x >> 6;
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) s_part[wave][k] = v[k];
    }
    __syncthreads();
    uint64_t r = 0;
    if (threadIdx.x < static_cast<uint32_t>(K)) {
        const bool use_or = (or_mask >> threadIdx.x) & 1u;
#pragma unroll
        for (int w = 0; w < NWAVE; w++) {
            const uint64_t x = s_part[w][threadIdx.x];
            r = use_or ? (r | x) : (r + x);
        }
    }
    __syncthreads();  // s_part is free again
    return r;
}

// A set of used symbols (up to MAX_SYMS) as SYM_WORDS 64-bit words.
struct SymSet {
    uint64_t w[SYM_WORDS];
};

// The used symbols with a transition out of some state of S (nsym used
// symbols in all): the only symbols whose successor set of S can be non-empty.
__device__ __forceinline__ SymSet symbols_of(const QueryView &qv, uint32_t S, uint32_t nsym) {
    SymSet r;
#pragma unroll
    for (int k = 0; k < SYM_WORDS; k++) r.w[k] = 0;
    while (S) {
        const uint64_t *m = qv.symmask + (__ffs(S) - 1) * SYM_WORDS;
        S &= S - 1;
#pragma unroll
        for (int k = 0; k < SYM_WORDS; k++)
            if (static_cast<uint32_t>(k) * 64 < nsym) r.w[k] |= m[k];
    }
    return r;
}

// Removes the lowest symbol of r and returns it, or ~0u when r is empty.
__device__ __forceinline__ uint32_t symbol_pop(SymSet &r) {
    uint32_t out = ~0u;
    bool found = false;
#pragma unroll
    for (int k = 0; k < SYM_WORDS; k++) {
        const bool here = !found && r.w[k] != 0;
        if (here) {
            out = static_cast<uint32_t>(k) * 64 +
                  static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(r.w[k]))) - 1;
            r.w[k] &= r.w[k] - 1;
        }
        found = found || here;
    }
    return out;
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

__device__ __forceinline__ uint32_t aload(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Row of vertex v in one (direction, label) of the store: returns false when
// v has no neighbours there, else the neighbour range [beg, end).
__device__ __forceinline__ bool row_range(const GraphView &g, const RankWordD &rw, uint64_t rbase, uint32_t v,
                                          uint32_t &beg, uint32_t &end) {
    const uint64_t bit = 1ull << (v & 63);
    if (!(rw.bits & bit)) return false;
    const uint64_t row = rbase + rw.rank + static_cast<uint32_t>(__popcll(rw.bits & (bit - 1)));
    beg = g.rowptr[row];
    end = g.rowptr[row + 1];
    return true;
}

// ------------------------------------------------------------ grid barrier
// Two-level barrier for the persistent kernels, whose grids are sized to be
// resident at once. Each XCD has its own L2. Workgroups first meet on a
// per-XCD counter; their stores are already in that XCD's L2 (every wave
// waits for its memory operations first). The last one on an XCD writes the
// L2 back once (device-scope release), meets the other XCDs' leaders on a
// global counter, invalidates its L2 (device-scope acquire) and releases the
// XCD's other workgroups, whose reads of data written during the launch are
// device-scope loads. Counters only grow within a launch (barrier k
// completes at k * members) and start at zero (the host clears the block
// before a launch; a single-query launch clears the next one's block). A wait longer
// than BARRIER_TIMEOUT ticks of the 100 MHz wall clock sets `abort`, and
// every workgroup leaves the kernel at its next barrier, so a workgroup that
// never becomes resident ends the launch instead of hanging it.
constexpr uint64_t BARRIER_TIMEOUT = 5ull * 100000000ull;  // 5 s

struct BarCtx {
    uint32_t xcd;    // this workgroup's XCD
    uint32_t per;    // workgroups on that XCD
    uint32_t nxcd;   // XCDs with workgroups
    uint32_t k;      // barriers passed
};

__device__ __forceinline__ uint32_t xcc_id() {
    // hardware register XCC_ID (id 20), bits [3:0]
    return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15u;
}

__device__ __forceinline__ bool spin_until_at_least(const GridBarrier *b, const uint32_t *ctr, uint32_t target) {
    const uint64_t t0 = wall_clock64();
    while (aload(ctr) < target) {
        if (aload(&b->abort)) return false;
        if (wall_clock64() - t0 > BARRIER_TIMEOUT) {
            __hip_atomic_store(const_cast<uint32_t *>(&b->abort), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// Registration at kernel start: every workgroup counts itself on its XCD
// (barrier_arrive_register), then waits until all have (barrier_wait_register)
// and learns how many share its XCD and how many XCDs take part. A workgroup
// may do work of its own between the two calls.
__device__ __forceinline__ void barrier_arrive_register(GridBarrier *b) {
    if (threadIdx.x == 0) {
        const uint32_t x = xcc_id();
        __hip_atomic_fetch_add(&b->reg[x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&b->nreg, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ inline bool barrier_wait_register(GridBarrier *b, BarCtx &c) {
    __shared__ uint32_t s_v[3];
    if (threadIdx.x == 0) {
        const uint32_t x = xcc_id();
        uint32_t ok = spin_until_at_least(b, &b->nreg, gridDim.x);
        // The two increments of a workgroup are independent relaxed atomics,
        // so the per-XCD counts may trail nreg: wait until they add up to the
        // grid as well (they only grow, and reach it once every workgroup's
        // first increment is visible), so that per and nxcd are final.
        uint32_t nx = 0;
        const uint64_t t0 = wall_clock64();
        while (ok) {
            uint32_t sum = 0;
            nx = 0;
            for (int i = 0; i < MAX_XCD; i++) {
                const uint32_t r = aload(&b->reg[i]);
                sum += r;
                nx += r ? 1u : 0u;
            }
            if (sum >= gridDim.x) break;
            if (aload(&b->abort)) ok = 0;
            else if (wall_clock64() - t0 > BARRIER_TIMEOUT) {
                __hip_atomic_store(&b->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
            } else {
                __builtin_amdgcn_s_sleep(1);
            }
        }
        s_v[0] = x;
        s_v[1] = aload(&b->reg[x]);
        s_v[2] = ok ? nx : 0u;
    }
    __syncthreads();
    c.xcd = s_v[0];
    c.per = s_v[1];
    c.nxcd = s_v[2];
    c.k = 0;
    return c.nxcd != 0;
}

__device__ inline bool barrier_register(GridBarrier *b, BarCtx &c) {
    barrier_arrive_register(b);
    return barrier_wait_register(b, c);
}

__device__ inline bool grid_barrier(GridBarrier *b, BarCtx &c) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads and stores are complete
    __syncthreads();
    c.k++;
    __shared__ uint32_t s_ok;
    if (threadIdx.x == 0) {
        uint32_t ok = 1;
        const uint32_t a =
            __hip_atomic_fetch_add(&b->lcount[c.xcd][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == c.k * c.per - 1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t ga = __hip_atomic_fetch_add(&b->gcount, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ga == c.k * c.nxcd - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                __hip_atomic_store(&b->ggen, c.k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                ok = spin_until_at_least(b, &b->ggen, c.k);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_store(&b->lgen[c.xcd][0], c.k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // the leader has invalidated the XCD's L2; this compute unit's L1
            // may hold stale lines, which the persistent kernels never read:
            // their loads of data written during the launch are device-scope
            // (ldc, ld_state). The fence only orders the compiler's accesses.
            ok = spin_until_at_least(b, &b->lgen[c.xcd][0], c.k);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        if (aload(&b->abort)) ok = 0;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

}  // namespace rpq
