// A ragged fill that allocates no device memory, for callers that cannot
// allocate (tight serving loops, harnesses that forbid allocation).  It does
// what rng_ragged_create followed by rng_fill_ragged_u32 does, with the same
// kernels, but the plan's work items, jump tables, lane maps, row slots and
// chunk states live in `scratch`, a fixed device array of kScratchBytes that
// each device holds for the life of the process.  The plan is made on the
// host for every call.
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device with hipGetSymbolAddress (the device current)
// and only that address is handed to copies and kernels.  Calls are
// serialised per process and return when the fill is done, so two calls never
// share the array at once from this process; nothing in it has to start at
// zero (every word a kernel reads was written earlier in the same call).
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "rngx_internal.h"

namespace rngx {

namespace {

constexpr size_t kScratchBytes = 64ull << 20;  // 64 MiB per device
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;                        // one call at a time; guards g_ptr
uint8_t *g_ptr[kMaxDevices] = {nullptr};  // device address of `scratch`, per device

// The array's address on device `dev` (current).  Caller holds g_mu.
hipError_t scratch_ptr(int dev, uint8_t **p) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_ptr[dev]) {
        void *addr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = static_cast<uint8_t *>(addr);
    }
    *p = g_ptr[dev];
    return hipSuccess;
}

size_t up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

}  // namespace

rngx_status ragged_fill_noalloc(Gen *g, const uint64_t *offsets, uint64_t units, uint32_t *d_out, hipStream_t st) {
    // A bound on the plan's size before it is made (the plan of a huge list
    // would itself take a lot of host memory): chunks of ragged_chunk values
    // per stream, or for XS1024W at most one chunk per instance and per row.
    uint64_t bound = 0;
    if (g->kind == RNGX_XS1024W) {
        bound = units + static_cast<uint64_t>(kXsRowsPerCu) * std::max(g->n_cu, 1) + 1;
    } else {
        const uint64_t C = ragged_chunk(g->kind);
        for (uint64_t u = 0; u < units; ++u) bound += (offsets[u + 1] - offsets[u] + C - 1) / C;
    }
    if (bound * (sizeof(RaggedItem) + ragged_scratch_bytes(g->kind, 1)) > kScratchBytes)
        return fail(RNGX_E_OVERFLOW, "the request list needs about " + std::to_string(bound) +
                                         " chunks, more than the 64 MiB scratch holds");
    RaggedPlan plan;
    ragged_plan(g->kind, offsets, units, g->n_cu, &plan);
    const std::vector<RaggedItem> &items = plan.items;
    if (items.empty()) return RNGX_OK;
    std::vector<uint64_t> t64, lane;
    std::vector<uint32_t> t32;
    jump_table_gen(g, plan.step, plan.max_j + 1, &t64, &t32);
    if (ragged_lane_table(g->kind)) ragged_lane_maps(g, &lane);
    // layout: items | chunk states | t64 | t32 | lane maps | slots
    const size_t b_items = up(sizeof(RaggedItem) * items.size());
    const size_t b_state = up(ragged_scratch_bytes(g->kind, items.size()));
    const size_t b_t64 = up(8 * t64.size()), b_t32 = up(4 * t32.size());
    const size_t b_lane = up(8 * lane.size()), b_slots = up(4 * plan.slots.size());
    const size_t need = b_items + b_state + b_t64 + b_t32 + b_lane + b_slots;
    if (need > kScratchBytes)
        return fail(RNGX_E_OVERFLOW, "the request list needs " + std::to_string(need) +
                                         " bytes of staging, more than the 64 MiB scratch");

    std::lock_guard<std::mutex> lk(g_mu);
    uint8_t *base = nullptr;
    hipError_t e = scratch_ptr(g->device, &base);
    if (e != hipSuccess) return hip_fail(e, "scratch address lookup");
    Ragged r{};
    r.gen = g;
    r.n_items = items.size();
    r.total = offsets[units];
    r.step = plan.step;
    r.n_slots = plan.slots.empty() ? 0 : static_cast<uint32_t>(plan.slots.size() - 1);
    size_t off = 0;
    r.d_items = reinterpret_cast<RaggedItem *>(base + off); off += b_items;
    r.d_scratch = base + off; off += b_state;
    r.d_t64 = t64.empty() ? nullptr : reinterpret_cast<uint64_t *>(base + off); off += b_t64;
    r.d_t32 = t32.empty() ? nullptr : reinterpret_cast<uint32_t *>(base + off); off += b_t32;
    r.d_lane = lane.empty() ? nullptr : reinterpret_cast<uint64_t *>(base + off); off += b_lane;
    r.d_slots = plan.slots.empty() ? nullptr : reinterpret_cast<uint32_t *>(base + off);
    e = hipMemcpyAsync(r.d_items, items.data(), sizeof(RaggedItem) * items.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && r.d_t64) e = hipMemcpyAsync(r.d_t64, t64.data(), 8 * t64.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && r.d_t32) e = hipMemcpyAsync(r.d_t32, t32.data(), 4 * t32.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && r.d_lane) e = hipMemcpyAsync(r.d_lane, lane.data(), 8 * lane.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && r.d_slots)
        e = hipMemcpyAsync(r.d_slots, plan.slots.data(), 4 * plan.slots.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_ragged(&r, d_out, st);
    // the host arrays are freed on return and the next call reuses the array
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "ragged fill from the static scratch");
    return RNGX_OK;
}

}  // namespace rngx
