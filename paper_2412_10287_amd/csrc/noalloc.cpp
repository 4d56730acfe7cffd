// rpq_multi_source_noalloc: the stacked multi-source traversal of
// rpq_multi_source with all of its per-call device state (frontier, visited
// and candidate rows, queues, work items, tile index, level records, grid
// barrier, status and counter words, query constants, the batch's sources and,
// for host output, the result bitmaps) in one fixed array of device memory
// that the library owns, so the call allocates nothing. The graph store and
// the handle's pinned staging buffer, both made by rpq_graph_load, are used
// as they are.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>

#include "api_internal.h"
#include "trace.h"
#include "stacked.h"

using namespace rpq;

namespace {

// The array itself (RPQ_NOALLOC_SCRATCH_BYTES) lives in stacked.hip, beside
// the kernels that use it. Every GPU the library runs on holds its own copy
// (at its own address) from the first call on that GPU until the process
// ends.
constexpr size_t SCRATCH_BYTES = RPQ_NOALLOC_SCRATCH_BYTES;

constexpr int MAX_DEVICES = 64;

// Per device: the array's device address (noalloc_scratch_address, with that
// device current), the stacked kernel's co-resident grids, and a lock: calls
// on one GPU share its array, so they run one at a time in this process.
struct DevScratch {
    std::mutex mu;
    bool ready = false;
    uint8_t *ptr = nullptr;
    int grid[2][17] = {{0}};
};
DevScratch g_dev[MAX_DEVICES];

// Once per device, with that device current.
rpq_status setup(DevScratch &d) {
    void *ptr = nullptr;
    const hipError_t e = noalloc_scratch_address(&ptr);
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    for (int G : {1, 2, 4, 8, 16}) {
        d.grid[0][G] = stacked_grid(G, 8);
        d.grid[1][G] = stacked_grid(G, 32);
    }
    d.ptr = static_cast<uint8_t *>(ptr);
    d.ready = true;
    return RPQ_OK;
}

}  // namespace

rpq_status rpq_multi_source_noalloc(rpq_graph *g, const rpq_nfa *n, const int32_t *sources, int32_t n_sources,
                                    uint64_t *out_bitmaps, uint32_t flags, rpq_stats *stats) {
    TraceRange tr_("rpq_multi_source_noalloc");
    if (!g) return fail(RPQ_EINVAL, "rpq_multi_source_noalloc: NULL argument");
    if (g->device < 0 || g->device >= MAX_DEVICES)
        return fail(RPQ_EINVAL, "rpq_multi_source_noalloc: device %d beyond the %d supported", g->device, MAX_DEVICES);
    DevScratch &d = g_dev[g->device];
    std::lock_guard<std::mutex> lk(d.mu);
    {
        const hipError_t e = hipSetDevice(g->device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    }
    if (!d.ready) {
        const rpq_status st = setup(d);
        if (st != RPQ_OK) return st;
    }
    StackArena ar;
    ar.base = d.ptr;
    ar.bytes = SCRATCH_BYTES;
    memcpy(ar.grid, d.grid, sizeof ar.grid);
    return stacked_run(g, n, sources, n_sources, out_bitmaps, flags, stats, "rpq_multi_source_noalloc", &ar);
}
