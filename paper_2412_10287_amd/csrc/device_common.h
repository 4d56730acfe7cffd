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

}  // namespace rpq
