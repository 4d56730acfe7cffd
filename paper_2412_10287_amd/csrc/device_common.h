// Device helpers shared by the single-query and multi-query kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "rpq_internal.h"

namespace rpq {

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
// Two-level barrier for the persistent kernel (every workgroup is resident:
// cooperative launch). Each XCD has its own L2. Workgroups first meet on a
// per-XCD counter; their stores are already in that XCD's L2 (every wave
// waits for its memory operations first). The last one on an XCD writes the
// L2 back once (device-scope release) and meets the other XCDs' leaders on a
// global counter; then every workgroup drops stale cached lines (device-scope
// acquire). Counters only grow within a launch (barrier k completes at
// k * members), and the host zeroes them before each launch. A wait longer
// than BARRIER_TIMEOUT ticks of the 100 MHz wall clock sets `abort`, and
// every workgroup leaves the kernel at its next barrier.
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

// Registration at kernel start: every workgroup counts itself on its XCD.
__device__ inline bool barrier_register(GridBarrier *b, BarCtx &c) {
    __shared__ uint32_t s_v[3];
    if (threadIdx.x == 0) {
        const uint32_t x = xcc_id();
        __hip_atomic_fetch_add(&b->reg[x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&b->nreg, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t ok = spin_until_at_least(b, &b->nreg, gridDim.x);
        uint32_t nx = 0;
        for (int i = 0; i < MAX_XCD; i++) nx += aload(&b->reg[i]) ? 1u : 0u;
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
            ok = spin_until_at_least(b, &b->lgen[c.xcd][0], c.k);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (aload(&b->abort)) ok = 0;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

}  // namespace rpq
