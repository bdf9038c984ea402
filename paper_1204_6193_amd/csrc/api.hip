// C-ABI entry points of rngx (declared and documented in include/rngx.h).
//
// Every entry point validates its arguments completely before touching the
// device; on error it returns a negative status with a thread-local message
// and modifies nothing.  Live handles are kept in a registry so that a
// stale or foreign handle is reported instead of dereferenced.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_set>
#include <vector>

#include "rngx_internal.h"

namespace rngx {

namespace {

constexpr uint64_t kGenMagic = 0x52474E5847454E31ull;    // "RGNXGEN1"
constexpr uint64_t kIsingMagic = 0x52474E584953474Eull;  // "RGNXISGN"
constexpr uint64_t kBatchMagic = 0x52474E5842415443ull;  // "RGNXBATC"
constexpr uint64_t kRaggedMagic = 0x52474E5852414747ull; // "RGNXRAGG"
constexpr uint64_t kMaxStreams = 1ull << 36;
constexpr uint32_t kMaxL = 16384;  // |E| <= 2 L^2 must fit int32

thread_local std::string g_error;
std::mutex g_mu;
std::unordered_set<const void *> g_live;

void reg(const void *p) { std::lock_guard<std::mutex> l(g_mu); g_live.insert(p); }
void unreg(const void *p) { std::lock_guard<std::mutex> l(g_mu); g_live.erase(p); }
bool live(const void *p) { std::lock_guard<std::mutex> l(g_mu); return p && g_live.count(p); }

// Makes the handle's device current for the scope of a call.
struct DeviceScope {
    int prev = -1, want;
    explicit DeviceScope(int dev) : want(dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != want) (void)hipSetDevice(want);
    }
    ~DeviceScope() { if (prev >= 0 && prev != want) (void)hipSetDevice(prev); }
};

bool mul_overflows(uint64_t a, uint64_t b, uint64_t *out) { return __builtin_mul_overflow(a, b, out); }

rngx_status check_gen(rngx_gen h, Gen **g) {
    if (!live(h)) return fail(RNGX_E_INVALID, "unknown or destroyed generator handle");
    *g = reinterpret_cast<Gen *>(h);
    if ((*g)->magic != kGenMagic) return fail(RNGX_E_INVALID, "corrupt generator handle");
    return RNGX_OK;
}

rngx_status check_ising(rngx_ising h, Ising **lat) {
    if (!live(h)) return fail(RNGX_E_INVALID, "unknown or destroyed lattice handle");
    *lat = reinterpret_cast<Ising *>(h);
    if ((*lat)->magic != kIsingMagic) return fail(RNGX_E_INVALID, "corrupt lattice handle");
    return RNGX_OK;
}

rngx_status check_batch(rngx_ising_batch h, IsingBatch **b) {
    if (!live(h)) return fail(RNGX_E_INVALID, "unknown or destroyed batch handle");
    *b = reinterpret_cast<IsingBatch *>(h);
    if ((*b)->magic != kBatchMagic) return fail(RNGX_E_INVALID, "corrupt batch handle");
    return RNGX_OK;
}

rngx_status check_ragged(rngx_ragged h, Ragged **r) {
    if (!live(h)) return fail(RNGX_E_INVALID, "unknown or destroyed ragged plan");
    *r = reinterpret_cast<Ragged *>(h);
    if ((*r)->magic != kRaggedMagic) return fail(RNGX_E_INVALID, "corrupt ragged plan");
    return RNGX_OK;
}

// The plan's device buffers.
void ragged_release(Ragged *r) {
    (void)hipFree(r->d_items);
    (void)hipFree(r->d_scratch);
    (void)hipFree(r->d_t64);
    (void)hipFree(r->d_t32);
    (void)hipFree(r->d_slots);
    (void)hipFree(r->d_lane);
    r->d_items = nullptr;
    r->d_scratch = nullptr;
    r->d_t64 = r->d_lane = nullptr;
    r->d_t32 = r->d_slots = nullptr;
    r->n_items = 0;
    r->n_slots = 0;
}

void free_ragged(Ragged *r) {
    ragged_release(r);
    r->magic = 0;
    delete r;
}

// (Re)builds r's plan from r->offsets under r->shape: work items, jump
// tables, lane maps, row slots and chunk-state scratch on the device.
rngx_status ragged_build(Ragged *r) {
    Gen *g = r->gen;
    ragged_release(r);
    const uint64_t units = r->offsets.size() - 1;
    RaggedPlan plan;
    ragged_plan(g->kind, r->offsets.data(), units, g->n_cu, &plan, r->shape);
    const std::vector<RaggedItem> &items = plan.items;
    if (items.size() > 0xFFFFFFFFull) return fail(RNGX_E_OVERFLOW, "too many chunks in one ragged plan");
    std::vector<uint64_t> t64;
    std::vector<uint32_t> t32;
    jump_table_gen(g, plan.step, plan.max_j + 1, &t64, &t32);
    r->total = r->offsets[units];
    r->step = plan.step;
    r->n_slots = plan.slots.empty() ? 0 : static_cast<uint32_t>(plan.slots.size() - 1);
    hipError_t e = hipSuccess;
    if (!items.empty()) {
        e = hipMalloc(&r->d_items, sizeof(RaggedItem) * items.size());
        if (e == hipSuccess && ragged_lane_table(g->kind)) {
            std::vector<uint64_t> lane;
            ragged_lane_maps(g, &lane);
            e = hipMalloc(&r->d_lane, 8 * lane.size());
            if (e == hipSuccess) e = hipMemcpy(r->d_lane, lane.data(), 8 * lane.size(), hipMemcpyHostToDevice);
        }
        if (e == hipSuccess && !plan.slots.empty()) e = hipMalloc(&r->d_slots, 4 * plan.slots.size());
        if (e == hipSuccess && !plan.slots.empty())
            e = hipMemcpy(r->d_slots, plan.slots.data(), 4 * plan.slots.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc(&r->d_scratch, ragged_scratch_bytes(g->kind, items.size()));
        if (e == hipSuccess && !t64.empty()) e = hipMalloc(&r->d_t64, 8 * t64.size());
        if (e == hipSuccess && !t32.empty()) e = hipMalloc(&r->d_t32, 4 * t32.size());
        if (e == hipSuccess)
            e = hipMemcpy(r->d_items, items.data(), sizeof(RaggedItem) * items.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !t64.empty()) e = hipMemcpy(r->d_t64, t64.data(), 8 * t64.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !t32.empty()) e = hipMemcpy(r->d_t32, t32.data(), 4 * t32.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        ragged_release(r);
        (void)hipGetLastError();
        return fail(RNGX_E_NOMEM, std::string("ragged plan allocation failed: ") + hipGetErrorString(e));
    }
    r->n_items = items.size();
    return RNGX_OK;
}

void free_batch(IsingBatch *b) {
    batch_release(b);
    delete[] b->lats;
    b->magic = 0;
    delete b;
}

rngx_status alloc_gen(rngx_kind kind, uint64_t S, Gen **out) {
    if (!kind_valid(kind)) return fail(RNGX_E_INVALID, "invalid generator kind " + std::to_string(kind));
    if (S == 0) return fail(RNGX_E_INVALID, "n_streams must be positive");
    if (S > kMaxStreams) return fail(RNGX_E_OVERFLOW, "n_streams exceeds 2^36");
    if (kind == RNGX_XS1024W && S % 32 != 0)
        return fail(RNGX_E_ALIGN, "XS1024W needs n_streams % 32 == 0 (32 lanes per 1024-bit instance)");
    if (kind == RNGX_MWC_DIFF && S > kMwcDiffMaxStreams)
        return fail(RNGX_E_OVERFLOW, "MWC_DIFF allows at most 2^21 streams (multipliers above 2^31)");
    if (is_lfg(kind) && S % kLfgLanes != 0)
        return fail(RNGX_E_ALIGN, "lagged Fibonacci kinds need n_streams % 1024 == 0 (1024 lanes per instance)");
    Gen *g = new Gen{};
    g->magic = kGenMagic;
    g->kind = kind;
    g->S = S;
    g->state_bytes = state_bytes(kind, S);
    if (is_sub_lcg(kind)) {
        affine_power(kind == RNGX_LCG32_SUB ? kLcg32A : kLcg64A, kind == RNGX_LCG32_SUB ? kLcg32C : kLcg64C, S,
                     &g->sub_a, &g->sub_c);
        if (kind == RNGX_LCG32_SUB) { g->sub_a &= 0xFFFFFFFFull; g->sub_c &= 0xFFFFFFFFull; }
    }
    if (hipGetDevice(&g->device) != hipSuccess) { delete g; return fail(RNGX_E_HIP, "hipGetDevice failed"); }
    hipError_t e = hipMalloc(&g->d_state, g->state_bytes);
    if (e != hipSuccess) {
        delete g;
        (void)hipGetLastError();
        return fail(RNGX_E_NOMEM, std::string("hipMalloc of generator state failed: ") + hipGetErrorString(e));
    }
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, g->device) != hipSuccess) n_cu = 0;
    e = fill_setup(g, n_cu);
    if (e == hipSuccess && is_lfg(kind)) e = hipMalloc(&g->d_aux, 4ull * lfg_lag_r(kind));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(g->d_state);
        (void)hipFree(g->d_ring);
        (void)hipFree(g->d_aux);
        delete g;
        return fail(RNGX_E_NOMEM, std::string("fill set-up failed: ") + hipGetErrorString(e));
    }
    *out = g;
    return RNGX_OK;
}

void free_gen(Gen *g) {
    if (!g) return;
    (void)hipFree(g->d_state);
    (void)hipFree(g->d_ring);
    (void)hipFree(g->d_aux);
    g->magic = 0;
    delete g;
}

rngx_status validate_image(rngx_kind kind, uint64_t S, const uint8_t *img) {
    if (kind == RNGX_XS1024W) {
        const uint32_t *W = reinterpret_cast<const uint32_t *>(img);
        for (uint64_t g = 0; g < S / 32; ++g) {
            uint32_t acc = 0;
            for (int i = 0; i < 32; ++i) acc |= W[32 * g + i];
            if (!acc) return fail(RNGX_E_STATE, "XS1024W instance " + std::to_string(g) + " is all-zero");
        }
    } else if (kind == RNGX_XORWOW) {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(img);
        for (uint64_t s = 0; s < S; ++s)
            if (!(p[s] | p[S + s] | p[2 * S + s] | p[3 * S + s] | p[4 * S + s]))
                return fail(RNGX_E_STATE, "XORWOW stream " + std::to_string(s) + " has all-zero xorshift words");
    } else if (kind == RNGX_MWC) {
        const uint64_t *y = reinterpret_cast<const uint64_t *>(img);
        for (uint64_t s = 0; s < S; ++s)
            if (y[s] == 0 || y[s] >= kMwcP)
                return fail(RNGX_E_STATE, "MWC stream " + std::to_string(s) + " is a fixed point (y = 0 or y >= p)");
    } else if (is_lfg(kind)) {
        const uint64_t r = lfg_lag_r(kind);
        const uint32_t *X = reinterpret_cast<const uint32_t *>(img);
        for (uint64_t g = 0; g < S / kLfgLanes; ++g) {
            uint32_t odd = 0;
            for (uint64_t j = 0; j < r; ++j) odd |= X[r * g + j] & 1u;
            if (!odd)
                return fail(RNGX_E_STATE, "lagged Fibonacci instance " + std::to_string(g) +
                                              " has only even words (its low bits would stay zero)");
        }
    } else if (kind == RNGX_MWC_DIFF) {
        const uint64_t *y = reinterpret_cast<const uint64_t *>(img);
        const uint32_t *a = reinterpret_cast<const uint32_t *>(img + 8 * S);
        if (!mwc_diff_multipliers_match(a, S))
            return fail(RNGX_E_STATE, "the image's multipliers are not this handle's (MWC_DIFF)");
        for (uint64_t s = 0; s < S; ++s)
            if (y[s] == 0 || y[s] >= (static_cast<uint64_t>(a[s]) << 32) - 1)
                return fail(RNGX_E_STATE, "MWC_DIFF stream " + std::to_string(s) + " is a fixed point (y = 0 or y >= p)");
    }
    return RNGX_OK;
}

rngx_status fill_common(rngx_gen h, void *d_out, uint64_t count, int mode, void *stream) {
    Gen *g;
    if (rngx_status s = check_gen(h, &g)) return s;
    if (!d_out) return fail(RNGX_E_INVALID, "output pointer is NULL");
    if (reinterpret_cast<uintptr_t>(d_out) % 16) return fail(RNGX_E_ALIGN, "output pointer must be 16-byte aligned");
    uint64_t n, bytes;
    if (mode != kOutXor && (mul_overflows(g->S, count, &n) || mul_overflows(n, 4, &bytes)))
        return fail(RNGX_E_OVERFLOW, "n_streams * count * 4 overflows 64 bits");
    if (count == 0 && mode != kOutXor) { clear_error(); return RNGX_OK; }
    DeviceScope ds(g->device);
    hipError_t e = launch_fill(g, d_out, count, mode, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "fill kernel launch");
    clear_error();
    return RNGX_OK;
}

}  // namespace

size_t state_bytes(rngx_kind kind, uint64_t S) {
    switch (kind) {
    case RNGX_LCG32: return 4 * S;
    case RNGX_LCG64: return 8 * S;
    case RNGX_MWC: return 8 * S;
    case RNGX_XORWOW: return 24 * S;
    case RNGX_PHILOX4X32_10:
    case RNGX_PHILOX4X32_7: return 16 * S;
    case RNGX_LCG32_SUB: return 4 * S + 8;
    case RNGX_LCG64_SUB: return 8 * S + 16;
    case RNGX_XS1024W: return 4 * S + 8 * (S / 32) + 4;
    case RNGX_MWC_DIFF: return 12 * S;
    case RNGX_LFG521: return 4 * 521 * (S / kLfgLanes);
    case RNGX_LFG1279: return 4 * 1279 * (S / kLfgLanes);
    }
    return 0;
}

bool kind_valid(int kind) { return kind >= RNGX_LCG32 && kind <= RNGX_MWC_DIFF; }

rngx_status fail(rngx_status st, const std::string &msg) { g_error = msg; return st; }
rngx_status hip_fail(hipError_t e, const char *what) {
    (void)hipGetLastError();
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return RNGX_E_HIP;
}
void clear_error() { g_error.clear(); }

}  // namespace rngx

using namespace rngx;

extern "C" {

const char *rngx_last_error(void) { return g_error.c_str(); }

rngx_status rng_create(rngx_kind kind, uint64_t n_streams, uint64_t seed, rngx_gen *out) {
    if (!out) return fail(RNGX_E_INVALID, "out is NULL");
    Gen *g;
    if (rngx_status s = alloc_gen(kind, n_streams, &g)) return s;
    hipError_t e = launch_seed(g, seed, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) { free_gen(g); return hip_fail(e, "seeding"); }
    reg(g);
    *out = reinterpret_cast<rngx_gen>(g);
    clear_error();
    return RNGX_OK;
}

rngx_status rng_create_substreams(rngx_kind kind, uint64_t n_streams, uint64_t seed, rngx_gen *out) {
    if (!out) return fail(RNGX_E_INVALID, "out is NULL");
    if (kind != RNGX_XS1024W) return fail(RNGX_E_INVALID, "sub-stream seeding is defined for XS1024W only");
    Gen *g;
    if (rngx_status s = alloc_gen(kind, n_streams, &g)) return s;
    hipError_t e = launch_seed(g, seed, nullptr);
    if (e == hipSuccess) e = launch_substreams(g, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) { free_gen(g); return hip_fail(e, "sub-stream seeding"); }
    reg(g);
    *out = reinterpret_cast<rngx_gen>(g);
    clear_error();
    return RNGX_OK;
}

rngx_status rng_destroy(rngx_gen h) {
    Gen *g;
    if (rngx_status s = check_gen(h, &g)) return s;
    if (g->owner) return fail(RNGX_E_INVALID, "this generator belongs to a lattice; destroy the lattice instead");
    if (g->plans) return fail(RNGX_E_BUSY, "a ragged plan still holds this generator; destroy it first");
    DeviceScope ds(g->device);
    (void)hipDeviceSynchronize();
    unreg(g);
    free_gen(g);
    clear_error();
    return RNGX_OK;
}

rngx_status rng_info(rngx_gen h, rngx_kind *kind, uint64_t *n_streams) {
    Gen *g;
    if (rngx_status s = check_gen(h, &g)) return s;
    if (kind) *kind = g->kind;
    if (n_streams) *n_streams = g->S;
    clear_error();
    return RNGX_OK;
}

rngx_status rng_fill_u32(rngx_gen g, uint32_t *d_out, uint64_t count, void *stream) {
    return fill_common(g, d_out, count, kOutU32, stream);
}

rngx_status rng_fill_f32(rngx_gen g, float *d_out, uint64_t count, void *stream) {
    return fill_common(g, d_out, count, kOutF32, stream);
}

rngx_status rng_consume(rngx_gen g, uint32_t *d_xor, uint64_t count, void *stream) {
    return fill_common(g, d_xor, count, kOutXor, stream);
}

rngx_status rng_fill_configs(rngx_kind kind, rngx_fill_config *out, int32_t *n) {
    if (!kind_valid(kind)) return fail(RNGX_E_INVALID, "invalid generator kind " + std::to_string(kind));
    if (!n) return fail(RNGX_E_INVALID, "n is NULL");
    const rngx_fill_config *list;
    const int k = fill_configs(kind, &list);
    if (out)
        for (int i = 0; i < k; ++i) out[i] = list[i];
    *n = k;
    clear_error();
    return RNGX_OK;
}

rngx_status rng_set_fill_config(rngx_gen h, int32_t index) {
    Gen *g;
    if (rngx_status s = check_gen(h, &g)) return s;
    const rngx_fill_config *list;
    const int k = fill_configs(g->kind, &list);
    if (index < -1 || index >= k) return fail(RNGX_E_INVALID, "fill configuration index out of range");
    g->fill_cfg = index;
    clear_error();
    return RNGX_OK;
}

rngx_status rng_get_fill_config(rngx_gen h, int32_t *index) {
    Gen *g;
    if (rngx_status s = check_gen(h, &g)) return s;
    if (!index) return fail(RNGX_E_INVALID, "index is NULL");
    *index = g->fill_cfg >= 0 ? g->fill_cfg : fill_default(g->kind);
    clear_error();
    return RNGX_OK;
}

rngx_status rng_autotune_fill(rngx_gen h, uint32_t *d_out, uint64_t count, int32_t reps, float *ms_out, void *stream) {
    Gen *g;
    if (rngx_status s = check_gen(h, &g)) return s;
    if (!d_out) return fail(RNGX_E_INVALID, "output pointer is NULL");
    if (reinterpret_cast<uintptr_t>(d_out) % 16) return fail(RNGX_E_ALIGN, "output pointer must be 16-byte aligned");
    if (count == 0 || reps < 1) return fail(RNGX_E_INVALID, "count and reps must be positive");
    uint64_t n, bytes;
    if (mul_overflows(g->S, count, &n) || mul_overflows(n, 4, &bytes))
        return fail(RNGX_E_OVERFLOW, "n_streams * count * 4 overflows 64 bits");
    DeviceScope ds(g->device);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const rngx_fill_config *list;
    const int k = fill_configs(g->kind, &list);
    void *saved = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&saved, g->state_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RNGX_E_NOMEM, "device memory for the saved state");
    }
    e = hipMemcpyAsync(saved, g->d_state, g->state_bytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int best = -1;
    float best_ms = 0;
    for (int i = 0; i < k && e == hipSuccess; ++i) {
        g->fill_cfg = i;
        e = hipMemcpyAsync(g->d_state, saved, g->state_bytes, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = launch_fill(g, d_out, count, kOutU32, st);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_fill(g, d_out, count, kOutU32, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        ms /= static_cast<float>(reps);
        if (ms_out) ms_out[i] = ms;
        if (e == hipSuccess && (best < 0 || ms < best_ms)) {
            best = i;
            best_ms = ms;
        }
    }
    // the stream state as it was before the call
    if (e == hipSuccess) e = hipMemcpyAsync(g->d_state, saved, g->state_bytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    g->fill_cfg = best;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(saved);
    if (e != hipSuccess) {
        g->fill_cfg = -1;
        return hip_fail(e, "fill autotuning");
    }
    clear_error();
    return RNGX_OK;
}

rngx_status rng_skip(rngx_gen h, uint64_t n, void *stream) {
    Gen *g;
    if (rngx_status s = check_gen(h, &g)) return s;
    if (n == 0) { clear_error(); return RNGX_OK; }
    DeviceScope ds(g->device);
    hipError_t e = launch_skip(g, n, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "skip kernel launch");
    clear_error();
    return RNGX_OK;
}

rngx_status rng_ragged_create(rngx_gen h, const uint64_t *offsets, uint64_t n_offsets, rngx_ragged *out) {
    Gen *g;
    if (rngx_status s = check_gen(h, &g)) return s;
    if (!offsets || !out) return fail(RNGX_E_INVALID, "NULL argument");
    if (is_lfg(g->kind)) return fail(RNGX_E_INVALID, "ragged fills do not take lagged Fibonacci kinds");
    const uint64_t units = g->kind == RNGX_XS1024W ? g->S / 32 : g->S;
    if (n_offsets != units + 1)
        return fail(RNGX_E_INVALID, "need " + std::to_string(units + 1) + " offsets, got " + std::to_string(n_offsets));
    for (uint64_t u = 0; u < units; ++u)
        if (offsets[u + 1] < offsets[u]) return fail(RNGX_E_INVALID, "offsets decrease at " + std::to_string(u));
    uint64_t bytes;
    if (mul_overflows(offsets[units], 4, &bytes)) return fail(RNGX_E_OVERFLOW, "output size overflows");
    DeviceScope ds(g->device);
    Ragged *r = new Ragged{};
    r->magic = kRaggedMagic;
    r->gen = g;
    r->shape = 0;
    r->offsets.assign(offsets, offsets + units + 1);
    if (rngx_status st = ragged_build(r)) {
        const std::string msg = g_error;
        free_ragged(r);
        return fail(st, msg);
    }
    ++g->plans;
    reg(r);
    *out = reinterpret_cast<rngx_ragged>(r);
    clear_error();
    return RNGX_OK;
}

rngx_status rng_fill_ragged_u32_noalloc(rngx_gen h, const uint64_t *offsets, uint64_t n_offsets, uint32_t *d_out,
                                        void *stream) {
    Gen *g;
    if (rngx_status s = check_gen(h, &g)) return s;
    if (!offsets) return fail(RNGX_E_INVALID, "offsets is NULL");
    if (is_lfg(g->kind)) return fail(RNGX_E_INVALID, "ragged fills do not take lagged Fibonacci kinds");
    const uint64_t units = g->kind == RNGX_XS1024W ? g->S / 32 : g->S;
    if (n_offsets != units + 1)
        return fail(RNGX_E_INVALID, "need " + std::to_string(units + 1) + " offsets, got " + std::to_string(n_offsets));
    for (uint64_t u = 0; u < units; ++u)
        if (offsets[u + 1] < offsets[u]) return fail(RNGX_E_INVALID, "offsets decrease at " + std::to_string(u));
    uint64_t bytes;
    if (mul_overflows(offsets[units], 4, &bytes)) return fail(RNGX_E_OVERFLOW, "output size overflows");
    if (!d_out && offsets[units]) return fail(RNGX_E_INVALID, "output pointer is NULL");
    if (reinterpret_cast<uintptr_t>(d_out) % 4) return fail(RNGX_E_ALIGN, "output must be 4-byte aligned");
    DeviceScope ds(g->device);
    if (rngx_status s = ragged_fill_noalloc(g, offsets, units, d_out, static_cast<hipStream_t>(stream))) return s;
    clear_error();
    return RNGX_OK;
}

rngx_status rng_fill_ragged_u32(rngx_ragged h, uint32_t *d_out, void *stream) {
    Ragged *r;
    if (rngx_status s = check_ragged(h, &r)) return s;
    if (!d_out && r->total) return fail(RNGX_E_INVALID, "output pointer is NULL");
    if (reinterpret_cast<uintptr_t>(d_out) % 4) return fail(RNGX_E_ALIGN, "output must be 4-byte aligned");
    if (r->total && !r->d_items) return fail(RNGX_E_HIP, "the plan was lost by a failed re-plan; set a shape again");
    DeviceScope ds(r->gen->device);
    hipError_t e = launch_ragged(r, d_out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "ragged fill launch");
    clear_error();
    return RNGX_OK;
}

rngx_status rng_ragged_shapes(rngx_kind kind, uint64_t *values, int32_t *n) {
    if (!n) return fail(RNGX_E_INVALID, "n is NULL");
    if (!kind_valid(kind) || is_lfg(kind)) return fail(RNGX_E_INVALID, "no ragged fills for this kind");
    if (values)
        for (int i = 0; i < kRaggedShapes; ++i) values[i] = ragged_shape_value(kind, i);
    *n = kRaggedShapes;
    clear_error();
    return RNGX_OK;
}

rngx_status rng_ragged_set_shape(rngx_ragged h, int32_t index) {
    Ragged *r;
    if (rngx_status s = check_ragged(h, &r)) return s;
    if (index < 0 || index >= kRaggedShapes) return fail(RNGX_E_INVALID, "shape index out of range");
    DeviceScope ds(r->gen->device);
    (void)hipDeviceSynchronize();  // no fill still reads the plan it replaces
    const int old = r->shape;
    r->shape = index;
    if (rngx_status st = ragged_build(r)) {
        const std::string msg = g_error;
        r->shape = old;
        (void)ragged_build(r);  // if this fails too, fills fail until a shape is set
        return fail(st, msg);
    }
    clear_error();
    return RNGX_OK;
}

rngx_status rng_ragged_get_shape(rngx_ragged h, int32_t *index) {
    Ragged *r;
    if (rngx_status s = check_ragged(h, &r)) return s;
    if (!index) return fail(RNGX_E_INVALID, "index is NULL");
    *index = r->shape;
    clear_error();
    return RNGX_OK;
}

rngx_status rng_ragged_autotune(rngx_ragged h, uint32_t *d_out, int32_t reps, float *ms_out, void *stream) {
    Ragged *r;
    if (rngx_status s = check_ragged(h, &r)) return s;
    if (reps < 1) return fail(RNGX_E_INVALID, "reps must be positive");
    if (!d_out && r->total) return fail(RNGX_E_INVALID, "output pointer is NULL");
    if (reinterpret_cast<uintptr_t>(d_out) % 4) return fail(RNGX_E_ALIGN, "output must be 4-byte aligned");
    Gen *g = r->gen;
    DeviceScope ds(g->device);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    void *saved = nullptr;
    hipError_t e = hipMalloc(&saved, g->state_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RNGX_E_NOMEM, "device memory for the saved stream states");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipDeviceSynchronize();  // no earlier fill, on any stream, still reads the plan
    if (e == hipSuccess) e = hipMemcpy(saved, g->d_state, g->state_bytes, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int start_shape = r->shape;
    int best = -1;
    float best_ms = 0;
    rngx_status built = RNGX_OK;
    for (int i = 0; i < kRaggedShapes && e == hipSuccess && built == RNGX_OK; ++i) {
        r->shape = i;
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        if ((built = ragged_build(r)) != RNGX_OK) break;
        e = hipMemcpyAsync(g->d_state, saved, g->state_bytes, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = launch_ragged(r, d_out, st);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int k = 0; k < reps && e == hipSuccess; ++k) e = launch_ragged(r, d_out, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        ms /= static_cast<float>(reps);
        if (ms_out) ms_out[i] = ms;
        if (e == hipSuccess && (best < 0 || ms < best_ms)) {
            best = i;
            best_ms = ms;
        }
    }
    const std::string build_msg = built != RNGX_OK ? g_error : std::string();
    // the fastest shape, and the streams as they were
    r->shape = best >= 0 ? best : start_shape;
    const hipError_t e_run = e;
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(g->d_state, saved, g->state_bytes, hipMemcpyDeviceToDevice);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(saved);
    const rngx_status rebuilt = ragged_build(r);
    if (built != RNGX_OK) return fail(built, build_msg);
    if (e_run != hipSuccess) return hip_fail(e_run, "ragged tuning run");
    if (e != hipSuccess) return hip_fail(e, "restoring the stream states");
    if (rebuilt != RNGX_OK) return rebuilt;
    clear_error();
    return RNGX_OK;
}

rngx_status rng_ragged_destroy(rngx_ragged h) {
    Ragged *r;
    if (rngx_status s = check_ragged(h, &r)) return s;
    DeviceScope ds(r->gen->device);
    (void)hipDeviceSynchronize();
    --r->gen->plans;
    unreg(r);
    free_ragged(r);
    clear_error();
    return RNGX_OK;
}

rngx_status rng_get_state(rngx_gen h, void *host_buf, size_t *bytes, void *stream) {
    Gen *g;
    if (rngx_status s = check_gen(h, &g)) return s;
    if (!bytes) return fail(RNGX_E_INVALID, "bytes is NULL");
    if (!host_buf) { *bytes = g->state_bytes; clear_error(); return RNGX_OK; }
    if (*bytes < g->state_bytes) return fail(RNGX_E_INVALID, "host buffer smaller than the state image");
    DeviceScope ds(g->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(host_buf, g->d_state, g->state_bytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "state copy to host");
    *bytes = g->state_bytes;
    clear_error();
    return RNGX_OK;
}

rngx_status rng_set_state(rngx_gen h, const void *host_buf, size_t bytes, void *stream) {
    Gen *g;
    if (rngx_status s = check_gen(h, &g)) return s;
    if (!host_buf) return fail(RNGX_E_INVALID, "host buffer is NULL");
    if (bytes != g->state_bytes)
        return fail(RNGX_E_STATE, "state image has " + std::to_string(bytes) + " bytes, expected " +
                                      std::to_string(g->state_bytes));
    if (rngx_status s = validate_image(g->kind, g->S, static_cast<const uint8_t *>(host_buf))) return s;
    if (is_sub_lcg(g->kind)) {
        uint64_t A, C;
        if (g->kind == RNGX_LCG32_SUB) {
            const uint32_t *p = static_cast<const uint32_t *>(host_buf);
            A = p[g->S]; C = p[g->S + 1];
        } else {
            const uint64_t *p = static_cast<const uint64_t *>(host_buf);
            A = p[g->S]; C = p[g->S + 1];
        }
        if (A != g->sub_a || C != g->sub_c)
            return fail(RNGX_E_STATE, "the image's S-step map is not this handle's (sub-stream LCG)");
    }
    DeviceScope ds(g->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(g->d_state, host_buf, bytes, hipMemcpyHostToDevice, st);
    // The caller may reuse host_buf on return: wait for the (pageable) copy.
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "state copy to device");
    clear_error();
    return RNGX_OK;
}

static void free_ising(Ising *lat) {
    (void)hipFree(lat->d_spins);
    (void)hipFree(lat->d_halo);
    (void)hipFree(lat->d_err);
    (void)hipFree(lat->d_partial);
    free_gen(lat->gen);
    lat->magic = 0;
    delete lat;
}

rngx_status ising_create(uint32_t L, rngx_kind kind, uint64_t seed, rngx_ising *out) {
    if (!out) return fail(RNGX_E_INVALID, "out is NULL");
    if (!kind_valid(kind)) return fail(RNGX_E_INVALID, "invalid generator kind " + std::to_string(kind));
    if (L < 16 || L % 16) return fail(RNGX_E_ALIGN, "L must be a multiple of 16 and at least 16");
    if (is_lfg(kind) && L % 64)
        return fail(RNGX_E_ALIGN, "lagged Fibonacci lattices need L % 64 == 0 (whole 1024-stream instances)");
    if (L > kMaxL) return fail(RNGX_E_OVERFLOW, "L must not exceed 16384 (int32 energies)");
    const uint64_t S = static_cast<uint64_t>(L) * L / 4;
    Gen *g;
    if (rngx_status s = alloc_gen(kind, S, &g)) return s;
    Ising *lat = new Ising{};
    lat->magic = kIsingMagic;
    lat->L = L;
    lat->device = g->device;
    lat->gen = g;
    g->owner = lat;
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, g->device) != hipSuccess) n_cu = 0;
    if (!ising_plan(L, kind, n_cu, &lat->plan)) lat->plan.strips = false;
    hipError_t e = hipMalloc(&lat->d_spins, static_cast<size_t>(L) * L);
    if (e == hipSuccess) e = hipMalloc(&lat->d_err, 4);
    if (e == hipSuccess && lat->plan.strips && lat->plan.nwg > 1) {
        e = hipMalloc(&lat->d_halo, static_cast<size_t>(8) * lat->plan.nwg * L);
        lat->halo_nwg = lat->plan.nwg;
    }
    // partials of the per-pass path (lagged Fibonacci multi-hit sweeps take it under any plan)
    if (e == hipSuccess && (!lat->plan.strips || is_lfg(kind))) e = hipMalloc(&lat->d_partial, 4 * ising_partials(L));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_ising(lat);
        return fail(RNGX_E_NOMEM, "device allocation for the lattice failed");
    }
    e = launch_seed(g, seed, nullptr);
    if (e == hipSuccess) e = launch_hot_start(lat, seed, nullptr);
    if (e == hipSuccess) e = launch_zero(lat->d_err, 1, nullptr);
    if (e == hipSuccess && lat->d_halo)  // tag 0 matches no pass
        e = launch_zero(reinterpret_cast<uint32_t *>(lat->d_halo), 2ull * lat->plan.nwg * L, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        free_ising(lat);
        return hip_fail(e, "lattice initialisation");
    }
    reg(g);
    reg(lat);
    *out = reinterpret_cast<rngx_ising>(lat);
    clear_error();
    return RNGX_OK;
}

rngx_status ising_sweep_hits(rngx_ising h, double beta, uint64_t n_sweeps, uint32_t hits, int32_t *d_trace,
                             void *stream) {
    Ising *lat;
    if (rngx_status s = check_ising(h, &lat)) return s;
    if (!std::isfinite(beta) || beta < 0) return fail(RNGX_E_INVALID, "beta must be finite and >= 0");
    if (hits < 1 || hits > (1u << 20)) return fail(RNGX_E_INVALID, "hits must be in 1 .. 2^20");
    if (d_trace && reinterpret_cast<uintptr_t>(d_trace) % 4) return fail(RNGX_E_ALIGN, "trace must be 4-byte aligned");
    if (n_sweeps == 0) { clear_error(); return RNGX_OK; }
    DeviceScope ds(lat->device);
    hipError_t e = launch_ising(lat, beta, n_sweeps, d_trace, static_cast<hipStream_t>(stream), hits);
    if (e != hipSuccess) return hip_fail(e, "Ising kernel launch");
    clear_error();
    return RNGX_OK;
}

rngx_status ising_sweep(rngx_ising h, double beta, uint64_t n_sweeps, int32_t *d_trace, void *stream) {
    return ising_sweep_hits(h, beta, n_sweeps, 1, d_trace, stream);
}

namespace {

constexpr int kMaxPlans = 15;

int plan_candidates(const Ising *lat, IsingPlan *list) {
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, lat->device) != hipSuccess) n_cu = 0;
    return ising_plan_list(lat->L, lat->gen->kind, n_cu, list, kMaxPlans);
}

// Switch the lattice to plan p (strips, or the per-pass path when
// !p.strips): waits for the device, sizes the buffers the plan needs and
// clears the halo tags.
hipError_t apply_plan(Ising *lat, const IsingPlan &p) {
    hipError_t e = hipDeviceSynchronize();
    const uint64_t L = lat->L;
    if (e == hipSuccess && p.strips && p.nwg > 1 && p.nwg > lat->halo_nwg) {
        (void)hipFree(lat->d_halo);
        lat->d_halo = nullptr;
        lat->halo_nwg = 0;
        e = hipMalloc(&lat->d_halo, 8ull * p.nwg * L);
        if (e == hipSuccess) lat->halo_nwg = p.nwg;
    }
    if (e == hipSuccess && (!p.strips || is_lfg(lat->gen->kind)) && !lat->d_partial)
        e = hipMalloc(&lat->d_partial, 4 * ising_partials(lat->L));
    if (e == hipSuccess && lat->d_halo)
        e = launch_zero(reinterpret_cast<uint32_t *>(lat->d_halo), 2ull * lat->halo_nwg * L, nullptr);
    if (e == hipSuccess) e = launch_zero(lat->d_err, 1, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return e;
    lat->plan = p;
    lat->epoch = 0;
    return hipSuccess;
}

}  // namespace

rngx_status ising_plans(rngx_ising h, uint32_t *strips_out, int32_t *n) {
    Ising *lat;
    if (rngx_status s = check_ising(h, &lat)) return s;
    if (!n) return fail(RNGX_E_INVALID, "n is NULL");
    DeviceScope ds(lat->device);
    IsingPlan list[kMaxPlans];
    const int k = plan_candidates(lat, list);
    if (strips_out) {
        for (int i = 0; i < k; ++i) strips_out[i] = list[i].nwg;
        strips_out[k] = 0;
    }
    *n = k + 1;
    clear_error();
    return RNGX_OK;
}

rngx_status ising_set_plan(rngx_ising h, uint32_t strips) {
    Ising *lat;
    if (rngx_status s = check_ising(h, &lat)) return s;
    DeviceScope ds(lat->device);
    IsingPlan p{};
    if (strips) {
        IsingPlan list[kMaxPlans];
        const int k = plan_candidates(lat, list);
        int i = 0;
        while (i < k && list[i].nwg != strips) ++i;
        if (i == k) return fail(RNGX_E_INVALID, "no strip plan with that many strips fits this lattice");
        p = list[i];
    }
    if (hipError_t e = apply_plan(lat, p)) return hip_fail(e, "switching the lattice's plan");
    clear_error();
    return RNGX_OK;
}

rngx_status ising_autotune(rngx_ising h, double beta, uint64_t n_sweeps, int32_t reps, float *ms_out, void *stream) {
    Ising *lat;
    if (rngx_status s = check_ising(h, &lat)) return s;
    if (!std::isfinite(beta) || beta < 0) return fail(RNGX_E_INVALID, "beta must be finite and >= 0");
    if (n_sweeps == 0 || reps < 1) return fail(RNGX_E_INVALID, "n_sweeps and reps must be positive");
    DeviceScope ds(lat->device);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    IsingPlan list[kMaxPlans + 1];
    const int k = plan_candidates(lat, list);
    list[k] = IsingPlan{};  // the per-pass path
    const size_t sbytes = static_cast<size_t>(lat->L) * lat->L, gbytes = lat->gen->state_bytes;
    void *saved_spins = nullptr, *saved_state = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&saved_spins, sbytes);
    if (e == hipSuccess) e = hipMalloc(&saved_state, gbytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(saved_spins);
        return fail(RNGX_E_NOMEM, "device memory for the saved lattice");
    }
    e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(saved_spins, lat->d_spins, sbytes, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(saved_state, lat->gen->d_state, gbytes, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int best = -1;
    float best_ms = 0;
    for (int i = 0; i <= k && e == hipSuccess; ++i) {
        e = apply_plan(lat, list[i]);
        if (e == hipSuccess) e = hipMemcpyAsync(lat->d_spins, saved_spins, sbytes, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(lat->gen->d_state, saved_state, gbytes, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = launch_ising(lat, beta, n_sweeps, nullptr, st);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_ising(lat, beta, n_sweeps, nullptr, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        ms /= static_cast<float>(reps);
        if (ms_out) ms_out[i] = ms;
        if (e == hipSuccess && (best < 0 || ms < best_ms)) {
            best = i;
            best_ms = ms;
        }
    }
    // the best plan, and the lattice and its streams as they were
    if (e == hipSuccess) e = apply_plan(lat, list[best]);
    if (e == hipSuccess) e = hipMemcpy(lat->d_spins, saved_spins, sbytes, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(lat->gen->d_state, saved_state, gbytes, hipMemcpyDeviceToDevice);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(saved_spins);
    (void)hipFree(saved_state);
    if (e != hipSuccess) return hip_fail(e, "Ising autotuning");
    clear_error();
    return RNGX_OK;
}

rngx_status ising_info(rngx_ising h, uint32_t *L, rngx_kind *kind, uint32_t *strips) {
    Ising *lat;
    if (rngx_status s = check_ising(h, &lat)) return s;
    if (L) *L = lat->L;
    if (kind) *kind = lat->gen->kind;
    if (strips) *strips = lat->plan.strips ? lat->plan.nwg : 0;
    clear_error();
    return RNGX_OK;
}

rngx_status ising_spins(rngx_ising h, int8_t **d_spins) {
    Ising *lat;
    if (rngx_status s = check_ising(h, &lat)) return s;
    if (!d_spins) return fail(RNGX_E_INVALID, "d_spins is NULL");
    *d_spins = lat->d_spins;
    clear_error();
    return RNGX_OK;
}

rngx_status ising_get_spins(rngx_ising h, int8_t *host_spins, void *stream) {
    Ising *lat;
    if (rngx_status s = check_ising(h, &lat)) return s;
    if (!host_spins) return fail(RNGX_E_INVALID, "host_spins is NULL");
    DeviceScope ds(lat->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n = static_cast<size_t>(lat->L) * lat->L;
    uint32_t err = 0;
    hipError_t e = hipMemcpyAsync(host_spins, lat->d_spins, n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&err, lat->d_err, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "spin copy to host");
    if (err) return fail(RNGX_E_HIP, "a strip gave up waiting for its neighbours; the lattice is invalid");
    clear_error();
    return RNGX_OK;
}

rngx_status ising_status(rngx_ising h, uint32_t *invalid, void *stream) {
    Ising *lat;
    if (rngx_status s = check_ising(h, &lat)) return s;
    if (!invalid) return fail(RNGX_E_INVALID, "invalid is NULL");
    DeviceScope ds(lat->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint32_t err = 0;
    hipError_t e = hipMemcpyAsync(&err, lat->d_err, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "status copy to host");
    *invalid = err ? 1 : 0;
    clear_error();
    return RNGX_OK;
}

rngx_status ising_set_spins(rngx_ising h, const int8_t *host_spins, void *stream) {
    Ising *lat;
    if (rngx_status s = check_ising(h, &lat)) return s;
    if (!host_spins) return fail(RNGX_E_INVALID, "host_spins is NULL");
    const size_t n = static_cast<size_t>(lat->L) * lat->L;
    for (size_t i = 0; i < n; ++i)
        if (host_spins[i] != 1 && host_spins[i] != -1)
            return fail(RNGX_E_STATE, "spin " + std::to_string(i) + " is neither +1 nor -1");
    DeviceScope ds(lat->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(lat->d_spins, host_spins, n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "spin copy to device");
    clear_error();
    return RNGX_OK;
}

rngx_status ising_rng(rngx_ising h, rngx_gen *g) {
    Ising *lat;
    if (rngx_status s = check_ising(h, &lat)) return s;
    if (!g) return fail(RNGX_E_INVALID, "g is NULL");
    *g = reinterpret_cast<rngx_gen>(lat->gen);
    clear_error();
    return RNGX_OK;
}

rngx_status ising_batch_create(const rngx_ising *lats, uint32_t n, const double *betas, const uint64_t *n_sweeps,
                               int32_t *const *d_traces, rngx_ising_batch *out) {
    if (!out || !lats || !betas || !n_sweeps) return fail(RNGX_E_INVALID, "NULL argument");
    if (n == 0) return fail(RNGX_E_INVALID, "a batch needs at least one lattice");
    std::vector<Ising *> members(n);
    std::unordered_set<const void *> seen;
    for (uint32_t i = 0; i < n; ++i) {
        if (rngx_status s = check_ising(lats[i], &members[i])) return s;
        if (!seen.insert(members[i]).second) return fail(RNGX_E_INVALID, "lattice " + std::to_string(i) + " repeats");
        if (members[i]->gen->kind != members[0]->gen->kind) return fail(RNGX_E_INVALID, "mixed generator kinds");
        if (is_lfg(members[i]->gen->kind)) return fail(RNGX_E_INVALID, "lagged Fibonacci lattices are not batched");
        if (members[i]->device != members[0]->device) return fail(RNGX_E_INVALID, "lattices on different devices");
        if (!std::isfinite(betas[i]) || betas[i] < 0) return fail(RNGX_E_INVALID, "beta must be finite and >= 0");
        if (d_traces && d_traces[i] && reinterpret_cast<uintptr_t>(d_traces[i]) % 4)
            return fail(RNGX_E_ALIGN, "traces must be 4-byte aligned");
    }
    DeviceScope ds(members[0]->device);
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, members[0]->device) != hipSuccess)
        return hip_fail(hipErrorInvalidDevice, "device query");
    IsingBatch *b = new IsingBatch{};
    b->magic = kBatchMagic;
    b->device = members[0]->device;
    b->kind = members[0]->gen->kind;
    b->n = n;
    b->n_cu = n_cu;
    b->shape = 0;
    b->lats = new Ising *[n];
    for (uint32_t i = 0; i < n; ++i) b->lats[i] = members[i];
    b->betas.assign(betas, betas + n);
    b->sweeps.assign(n_sweeps, n_sweeps + n);
    b->traces.assign(n, nullptr);
    if (d_traces) b->traces.assign(d_traces, d_traces + n);
    hipError_t e = batch_prepare(b, b->sweeps.data(), true);
    if (e != hipSuccess) {
        free_batch(b);
        return hip_fail(e, "batch preparation");
    }
    for (uint32_t i = 0; i < n; ++i) ++members[i]->batches;
    reg(b);
    *out = reinterpret_cast<rngx_ising_batch>(b);
    clear_error();
    return RNGX_OK;
}

rngx_status ising_batch_run(rngx_ising_batch h, void *stream) {
    IsingBatch *b;
    if (rngx_status s = check_batch(h, &b)) return s;
    DeviceScope ds(b->device);
    hipError_t e = launch_batch(b, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    clear_error();
    return RNGX_OK;
}

rngx_status ising_batch_status(rngx_ising_batch h, uint32_t *n_invalid, void *stream) {
    IsingBatch *b;
    if (rngx_status s = check_batch(h, &b)) return s;
    if (!n_invalid) return fail(RNGX_E_INVALID, "n_invalid is NULL");
    DeviceScope ds(b->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<uint32_t> err(b->n, 0);
    hipError_t e = hipSuccess;
    for (uint32_t i = 0; i < b->n && e == hipSuccess; ++i)
        e = hipMemcpyAsync(&err[i], b->lats[i]->d_err, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "status copy to host");
    uint32_t bad = 0;
    for (uint32_t v : err) bad += v ? 1 : 0;
    *n_invalid = bad;
    clear_error();
    return RNGX_OK;
}

rngx_status ising_batch_info(rngx_ising_batch h, uint32_t *n_items, uint32_t *resident, uint32_t *grid) {
    IsingBatch *b;
    if (rngx_status s = check_batch(h, &b)) return s;
    if (n_items) *n_items = b->n_items;
    if (resident) *resident = b->resident;
    if (grid) *grid = b->grid;
    clear_error();
    return RNGX_OK;
}

rngx_status ising_batch_shapes(rngx_batch_shape *out, int32_t *n) {
    if (!n) return fail(RNGX_E_INVALID, "n is NULL");
    if (out)
        for (int i = 0; i < kBatchShapes; ++i)
            out[i] = rngx_batch_shape{kBatchShape[i].threads, kBatchShape[i].sites_per_thread, kBatchShape[i].lds_cap};
    *n = kBatchShapes;
    clear_error();
    return RNGX_OK;
}

rngx_status ising_batch_set_shape(rngx_ising_batch h, int32_t index) {
    IsingBatch *b;
    if (rngx_status s = check_batch(h, &b)) return s;
    if (index < 0 || index >= kBatchShapes) return fail(RNGX_E_INVALID, "shape index out of range");
    DeviceScope ds(b->device);
    (void)hipDeviceSynchronize();  // no run of the old plan still reads its buffers
    const int old = b->shape;
    b->shape = index;
    hipError_t e = batch_prepare(b, b->sweeps.data(), true);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b->shape = old;
        (void)batch_prepare(b, b->sweeps.data(), true);  // if this fails too, runs fail until a shape is set
        (void)hipGetLastError();
        return hip_fail(e, "batch re-planning");
    }
    clear_error();
    return RNGX_OK;
}

rngx_status ising_batch_get_shape(rngx_ising_batch h, int32_t *index) {
    IsingBatch *b;
    if (rngx_status s = check_batch(h, &b)) return s;
    if (!index) return fail(RNGX_E_INVALID, "index is NULL");
    *index = b->shape;
    clear_error();
    return RNGX_OK;
}

rngx_status ising_batch_autotune(rngx_ising_batch h, uint64_t max_sweeps, int32_t reps, float *ms_out, void *stream) {
    IsingBatch *b;
    if (rngx_status s = check_batch(h, &b)) return s;
    if (max_sweeps == 0 || reps < 1) return fail(RNGX_E_INVALID, "max_sweeps and reps must be positive");
    DeviceScope ds(b->device);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    // Tuning runs: every replica's sweep count scaled by one factor so that
    // the longest runs max_sweeps (at least one sweep each), no traces.
    uint64_t top = 1;
    for (uint64_t v : b->sweeps) top = std::max(top, v);
    std::vector<uint64_t> tune(b->n);
    for (uint32_t i = 0; i < b->n; ++i)
        tune[i] = top <= max_sweeps ? b->sweeps[i]
                                    : std::max<uint64_t>(1, static_cast<uint64_t>(static_cast<double>(b->sweeps[i]) *
                                                                                  max_sweeps / top + 0.5));
    // every replica's spins, streams and status word, saved in one buffer
    std::vector<size_t> off(b->n + 1, 0);
    for (uint32_t i = 0; i < b->n; ++i) {
        const Ising *l = b->lats[i];
        off[i + 1] = off[i] + (static_cast<size_t>(l->L) * l->L + l->gen->state_bytes + 4 + 255) / 256 * 256;
    }
    uint8_t *saved = nullptr;
    hipError_t e = hipMalloc(&saved, off[b->n]);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RNGX_E_NOMEM, "device memory for the saved replicas");
    }
    auto copy_all = [&](bool save) {
        hipError_t r = hipSuccess;
        for (uint32_t i = 0; i < b->n && r == hipSuccess; ++i) {
            Ising *l = b->lats[i];
            const size_t sb = static_cast<size_t>(l->L) * l->L, gb = l->gen->state_bytes;
            uint8_t *p = saved + off[i];
            void *dev[3] = {l->d_spins, l->gen->d_state, l->d_err};
            const size_t at[3] = {0, sb, sb + gb}, len[3] = {sb, gb, 4};
            for (int k = 0; k < 3 && r == hipSuccess; ++k)
                r = save ? hipMemcpyAsync(p + at[k], dev[k], len[k], hipMemcpyDeviceToDevice, st)
                         : hipMemcpyAsync(dev[k], p + at[k], len[k], hipMemcpyDeviceToDevice, st);
        }
        return r;
    };
    const int start_shape = b->shape;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipDeviceSynchronize();  // no earlier run, on any stream, still reads the plan it replaces
    if (e == hipSuccess) e = copy_all(true);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int best = -1;
    float best_ms = 0;
    for (int i = 0; i < kBatchShapes && e == hipSuccess; ++i) {
        b->shape = i;
        e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = batch_prepare(b, tune.data(), false);
        if (e == hipSuccess) e = copy_all(false);
        if (e == hipSuccess) e = launch_batch(b, st);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_batch(b, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        ms /= static_cast<float>(reps);
        if (ms_out) ms_out[i] = ms;
        if (e == hipSuccess && (best < 0 || ms < best_ms)) {
            best = i;
            best_ms = ms;
        }
    }
    // the fastest shape with the real sweep counts and traces, and the
    // replicas as they were
    b->shape = best >= 0 ? best : start_shape;
    const hipError_t e_run = e;
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = copy_all(false);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(saved);
    const hipError_t e_plan = batch_prepare(b, b->sweeps.data(), true);
    if (e_run != hipSuccess) return hip_fail(e_run, "batch tuning run");
    if (e != hipSuccess) return hip_fail(e, "restoring the replicas");
    if (e_plan != hipSuccess) return hip_fail(e_plan, "batch re-planning");
    clear_error();
    return RNGX_OK;
}

rngx_status ising_batch_destroy(rngx_ising_batch h) {
    IsingBatch *b;
    if (rngx_status s = check_batch(h, &b)) return s;
    DeviceScope ds(b->device);
    (void)hipDeviceSynchronize();
    for (uint32_t i = 0; i < b->n; ++i) --b->lats[i]->batches;
    unreg(b);
    free_batch(b);
    clear_error();
    return RNGX_OK;
}

rngx_status ising_destroy(rngx_ising h) {
    Ising *lat;
    if (rngx_status s = check_ising(h, &lat)) return s;
    if (lat->batches) return fail(RNGX_E_BUSY, "a batch still holds this lattice; destroy the batch first");
    DeviceScope ds(lat->device);
    (void)hipDeviceSynchronize();
    unreg(lat);
    unreg(lat->gen);
    free_ising(lat);
    clear_error();
    return RNGX_OK;
}

rngx_status srv_create(const rngx_server_config *cfg, rngx_server *out) {
    if (!cfg || !out) return fail(RNGX_E_INVALID, "NULL argument");
    if (cfg->slots < 1 || cfg->max_inflight < 1) return fail(RNGX_E_INVALID, "slots and max_inflight must be >= 1");
    if (cfg->memory_budget == 0) return fail(RNGX_E_INVALID, "memory_budget must be positive");
    Server *s;
    if (rngx_status st = server_create(cfg, &s)) return st;
    reg(s);
    *out = reinterpret_cast<rngx_server>(s);
    clear_error();
    return RNGX_OK;
}

static rngx_status check_server(rngx_server h, Server **s) {
    if (!live(h)) return fail(RNGX_E_INVALID, "unknown or destroyed server");
    *s = reinterpret_cast<Server *>(h);
    return RNGX_OK;
}

rngx_status srv_submit_fill(rngx_server h, uint32_t client, rngx_kind kind, uint64_t count, int as_f32,
                            uint64_t *ticket) {
    Server *s;
    if (rngx_status st = check_server(h, &s)) return st;
    if (!ticket) return fail(RNGX_E_INVALID, "ticket is NULL");
    if (!kind_valid(kind) || is_sub_lcg(kind) || kind == RNGX_MWC_DIFF || is_lfg(kind))
        return fail(RNGX_E_INVALID, "invalid generator kind (sub-stream LCG, MWC_DIFF and LFG kinds are not served)");
    if (count == 0) return fail(RNGX_E_INVALID, "count must be positive");
    if (count > kMaxServedValues) return fail(RNGX_E_OVERFLOW, "count exceeds 2^28");
    if (rngx_status st = server_submit_fill(s, client, kind, count, as_f32, ticket)) return st;
    clear_error();
    return RNGX_OK;
}

rngx_status srv_submit_ising(rngx_server h, uint32_t client, rngx_kind kind, uint32_t L, double beta,
                             uint32_t n_sweeps, uint64_t *ticket) {
    Server *s;
    if (rngx_status st = check_server(h, &s)) return st;
    if (!ticket) return fail(RNGX_E_INVALID, "ticket is NULL");
    if (!kind_valid(kind) || is_sub_lcg(kind) || kind == RNGX_MWC_DIFF || is_lfg(kind))
        return fail(RNGX_E_INVALID, "invalid generator kind (sub-stream LCG, MWC_DIFF and LFG kinds are not served)");
    if (L < 16 || L % 16) return fail(RNGX_E_ALIGN, "L must be a multiple of 16 and at least 16");
    if (L > kMaxL) return fail(RNGX_E_OVERFLOW, "L must not exceed 16384");
    if (!std::isfinite(beta) || beta < 0) return fail(RNGX_E_INVALID, "beta must be finite and >= 0");
    if (rngx_status st = server_submit_ising(s, client, kind, L, beta, n_sweeps, ticket)) return st;
    clear_error();
    return RNGX_OK;
}

rngx_status srv_wait(rngx_server h, uint64_t ticket, double timeout_s, rngx_request_result *res) {
    Server *s;
    if (rngx_status st = check_server(h, &s)) return st;
    if (!res) return fail(RNGX_E_INVALID, "res is NULL");
    if (rngx_status st = server_wait(s, ticket, timeout_s, res)) return st;
    clear_error();
    return RNGX_OK;
}

rngx_status srv_wait_any(rngx_server h, double timeout_s, uint64_t *ticket, rngx_request_result *res) {
    Server *s;
    if (rngx_status st = check_server(h, &s)) return st;
    if (!res || !ticket) return fail(RNGX_E_INVALID, "NULL argument");
    if (rngx_status st = server_wait_any(s, timeout_s, ticket, res)) return st;
    clear_error();
    return RNGX_OK;
}

rngx_status srv_release(rngx_server h, uint64_t ticket) {
    Server *s;
    if (rngx_status st = check_server(h, &s)) return st;
    if (rngx_status st = server_release(s, ticket)) return st;
    clear_error();
    return RNGX_OK;
}

rngx_status srv_cancel(rngx_server h, uint64_t ticket) {
    Server *s;
    if (rngx_status st = check_server(h, &s)) return st;
    if (rngx_status st = server_cancel(s, ticket)) return st;
    clear_error();
    return RNGX_OK;
}

static rngx_status check_served_kind(rngx_kind kind) {
    if (!kind_valid(kind) || is_sub_lcg(kind) || kind == RNGX_MWC_DIFF || is_lfg(kind))
        return fail(RNGX_E_INVALID, "invalid generator kind (sub-stream LCG, MWC_DIFF and LFG kinds are not served)");
    return RNGX_OK;
}

rngx_status srv_get_client_state(rngx_server h, uint32_t client, rngx_kind kind, void *host_buf, size_t *bytes) {
    Server *s;
    if (rngx_status st = check_server(h, &s)) return st;
    if (rngx_status st = check_served_kind(kind)) return st;
    if (!bytes) return fail(RNGX_E_INVALID, "bytes is NULL");
    const size_t need = server_client_state_bytes(kind);
    if (!host_buf) { *bytes = need; clear_error(); return RNGX_OK; }
    if (*bytes < need) return fail(RNGX_E_INVALID, "host buffer smaller than the client's state image");
    DeviceScope ds(server_device(s));
    if (rngx_status st = server_get_client_state(s, client, kind, host_buf)) return st;
    *bytes = need;
    clear_error();
    return RNGX_OK;
}

rngx_status srv_set_client_state(rngx_server h, uint32_t client, rngx_kind kind, const void *host_buf, size_t bytes) {
    Server *s;
    if (rngx_status st = check_server(h, &s)) return st;
    if (rngx_status st = check_served_kind(kind)) return st;
    if (!host_buf) return fail(RNGX_E_INVALID, "host buffer is NULL");
    const size_t need = server_client_state_bytes(kind);
    if (bytes != need)
        return fail(RNGX_E_STATE, "state image has " + std::to_string(bytes) + " bytes, expected " + std::to_string(need));
    const uint64_t S = kind == RNGX_XS1024W ? 32 : 1;
    if (rngx_status st = validate_image(kind, S, static_cast<const uint8_t *>(host_buf))) return st;
    DeviceScope ds(server_device(s));
    if (rngx_status st = server_set_client_state(s, client, kind, host_buf)) return st;
    clear_error();
    return RNGX_OK;
}

rngx_status srv_destroy(rngx_server h) {
    Server *s;
    if (rngx_status st = check_server(h, &s)) return st;
    unreg(s);
    server_destroy(s);
    clear_error();
    return RNGX_OK;
}

}  // extern "C"
