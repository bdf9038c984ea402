// Served form: a request loop with continuous batching.
//
// Requests (random-number fills and Ising jobs) are submitted from any host
// thread and stamped on arrival.  A worker thread admits them in arrival
// order as soon as the device-memory pool and the in-flight limit allow (a
// request that does not fit yet is passed by later ones of other (client,
// kind) pairs, at most kMaxBypass times, after which admission waits for
// memory to come back to it),
// launches their work on one of `slots` HIP streams, and detects completion
// with events, so requests that arrive while others run are started at once
// and overlap on the device.  Each (client, kind) keeps a resident generator
// whose requests always go to the same stream, so they run in submission
// order; different clients run concurrently.  Ising jobs use only paths
// whose workgroups never wait on each other (one workgroup per lattice, or
// one launch per colour pass), so concurrent jobs cannot depend on being
// co-resident.  No device allocation happens per request: outputs come from
// one pool allocated at creation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rngx_internal.h"

namespace rngx {

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over one device allocation.
class Pool {
  public:
    bool init(uint64_t bytes) {
        if (hipMalloc(&base_, bytes) != hipSuccess) { (void)hipGetLastError(); return false; }
        free_[0] = bytes;
        size_ = bytes;
        return true;
    }
    ~Pool() { if (base_) (void)hipFree(base_); }
    // Returns the offset, or UINT64_MAX if no block fits.
    uint64_t alloc(uint64_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const uint64_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_[off] = bytes;
            return off;
        }
        return UINT64_MAX;
    }
    void release(uint64_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return;
        uint64_t size = u->second;
        used_.erase(u);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + size) { size += next->second; next = free_.erase(next); }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) { prev->second += size; return; }
        }
        free_[off] = size;
    }
    uint8_t *ptr(uint64_t off) const { return static_cast<uint8_t *>(base_) + off; }
    uint64_t size() const { return size_; }

  private:
    void *base_ = nullptr;
    uint64_t size_ = 0;
    std::map<uint64_t, uint64_t> free_, used_;
};

uint64_t round16(uint64_t x) { return (x + 15) / 16 * 16; }

constexpr uint32_t kMaxBypass = 64;  // later requests that may pass one waiting for memory

}  // namespace

struct ServerRequest {
    uint64_t ticket;
    int type;  // 0 fill, 1 ising
    uint32_t client;
    rngx_kind kind;
    uint64_t count;  // fill: values requested
    int f32;
    uint32_t L, sweeps;
    double beta;
    uint64_t ising_index;  // this client's Ising job number
    Clock::time_point arrival, done_at;
    uint64_t bytes = 0, pool_off = UINT64_MAX;
    uint64_t n_values = 0;
    hipEvent_t ev = nullptr;
    int state = 0;  // 0 pending, 1 in flight, 2 done, 3 failed
    uint32_t bypassed = 0;  // later requests admitted while this one waited for memory
    // Ising job scratch descriptors (point into the pool)
    Gen job_gen{};
    Ising job_lat{};
};

// A (client, kind) generator: one stream (XS1024W: one instance), its state
// in two pool buffers used alternately, one per request.
struct ClientGen {
    rngx_kind kind;
    uint8_t *buf[2];
    int cur;
};

struct Server {
    uint64_t magic;
    rngx_server_config cfg;
    int device = 0, n_cu = 0;
    Pool pool;
    std::vector<hipStream_t> streams;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<ServerRequest>> pending;
    std::vector<std::shared_ptr<ServerRequest>> inflight;
    std::vector<std::shared_ptr<ServerRequest>> launching;  // admitted, being launched (lock released)
    std::unordered_map<uint64_t, std::shared_ptr<ServerRequest>> all;
    std::map<std::pair<uint32_t, int>, ClientGen *> gens;
    const uint64_t *t64[8] = {};  // per-kind jump tables for chunks of stream_fill_chunk(kind)
    const uint32_t *t32[8] = {};
    std::unordered_map<uint32_t, uint64_t> ising_count;
    std::deque<uint64_t> completed;  // finished tickets not yet returned by wait_any
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    std::vector<hipEvent_t> spare_events;
};

namespace {

uint64_t request_bytes(const Server *s, const ServerRequest &r) {
    if (r.type == 0) return 4 * r.count;
    const uint64_t L = r.L, S = L * L / 4;
    return round16(L * L) + round16(4ull * r.sweeps) + round16(state_bytes(r.kind, S)) + 4 * ising_partials(r.L);
}

hipEvent_t take_event(Server *s) {
    if (!s->spare_events.empty()) {
        hipEvent_t e = s->spare_events.back();
        s->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
    return e;
}

uint64_t unit_streams(rngx_kind kind) { return kind == RNGX_XS1024W ? 32 : 1; }

// Generator of (client, kind), created and seeded on first use: stream 0
// (instance 0) of rng_create(kind, 1 or 32, splitmix64 output 16 client +
// kind of the server seed).
ClientGen *client_gen(Server *s, uint32_t client, rngx_kind kind, hipStream_t st) {
    auto key = std::make_pair(client, static_cast<int>(kind));
    auto it = s->gens.find(key);
    if (it != s->gens.end()) return it->second;
    const uint64_t bytes = state_bytes(kind, unit_streams(kind));
    const uint64_t off = s->pool.alloc(2 * ((bytes + 255) / 256 * 256));  // held until the server is destroyed
    if (off == UINT64_MAX) return nullptr;
    ClientGen *c = new ClientGen{kind, {s->pool.ptr(off), s->pool.ptr(off + (bytes + 255) / 256 * 256)}, 0};
    Gen g{};
    g.kind = kind;
    g.S = unit_streams(kind);
    g.d_state = c->buf[0];
    g.state_bytes = bytes;
    if (launch_seed(&g, splitmix(s->cfg.seed, 16ull * client + kind), st) != hipSuccess) {
        s->pool.release(off);
        delete c;
        return nullptr;
    }
    s->gens[key] = c;
    return c;
}

hipStream_t stream_for(Server *s, uint32_t client, rngx_kind kind) {
    return s->streams[(static_cast<uint64_t>(client) * 7 + kind) % s->streams.size()];
}

// Launch a request's work (worker thread, lock not held; `c` is the
// client's generator for fills).  Returns false on failure.
bool launch_request(Server *s, ServerRequest &r, ClientGen *c) {
    hipStream_t st = stream_for(s, r.client, r.kind);
    uint8_t *base = s->pool.ptr(r.pool_off);
    if (r.type == 0) {
        if (!c) return false;
        r.n_values = r.count;
        if (launch_stream_fill(r.kind, c->buf[c->cur], c->buf[c->cur ^ 1], r.count, r.f32, s->t64[r.kind],
                               s->t32[r.kind], base, st) != hipSuccess)
            return false;
        c->cur ^= 1;  // requests of one client and kind are launched in order on one stream
    } else {
        const uint64_t L = r.L, S = L * L / 4;
        Gen &g = r.job_gen;
        Ising &lat = r.job_lat;
        g.kind = r.kind;
        g.S = S;
        g.device = s->device;
        g.state_bytes = state_bytes(r.kind, S);
        lat.L = r.L;
        lat.device = s->device;
        lat.gen = &g;
        lat.d_spins = reinterpret_cast<int8_t *>(base);
        int32_t *trace = reinterpret_cast<int32_t *>(base + round16(L * L));
        g.d_state = base + round16(L * L) + round16(4ull * r.sweeps);
        lat.d_partial = reinterpret_cast<int32_t *>(g.d_state + round16(g.state_bytes));
        // Multi-strip lattices need all their workgroups resident at once,
        // which concurrent requests could prevent: served jobs use one
        // workgroup (small L) or one launch per colour pass instead.
        IsingPlan plan{};
        if (!ising_plan(r.L, r.kind, s->n_cu, &plan) || plan.nwg != 1) plan = IsingPlan{};
        lat.plan = plan;
        // Ising job seed: splitmix64 output 2^62 + 2^24 client + job index.
        const uint64_t seed = splitmix(s->cfg.seed, (1ull << 62) + (static_cast<uint64_t>(r.client) << 24) + r.ising_index);
        r.n_values = L * L;
        if (launch_seed(&g, seed, st) != hipSuccess) return false;
        if (launch_hot_start(&lat, seed, st) != hipSuccess) return false;
        if (r.sweeps && launch_ising(&lat, r.beta, r.sweeps, trace, st) != hipSuccess) return false;
    }
    r.ev = take_event(s);
    if (!r.ev || hipEventRecord(r.ev, st) != hipSuccess) return false;
    return true;
}

void worker_loop(Server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        bool progress = false;
        // completions
        for (size_t i = 0; i < s->inflight.size();) {
            auto &r = s->inflight[i];
            const hipError_t q = hipEventQuery(r->ev);
            if (q == hipErrorNotReady) { ++i; continue; }
            r->done_at = Clock::now();
            r->state = q == hipSuccess ? 2 : 3;
            if (q != hipSuccess) (void)hipGetLastError();
            s->spare_events.push_back(r->ev);
            r->ev = nullptr;
            s->completed.push_back(r->ticket);
            s->inflight[i] = s->inflight.back();
            s->inflight.pop_back();
            progress = true;
        }
        if (progress) s->cv_done.notify_all();
        // admissions: the first pending request that fits, in arrival order,
        // never ahead of an earlier one of its own (client, kind) (its
        // stream's order) nor past one that has been passed kMaxBypass times
        while (!s->pending.empty() && s->inflight.size() < s->cfg.max_inflight) {
            std::shared_ptr<ServerRequest> r;
            std::vector<std::pair<uint32_t, int>> blocked;
            for (size_t i = 0; i < s->pending.size(); ++i) {
                auto &c = s->pending[i];
                const auto key = std::make_pair(c->client, static_cast<int>(c->kind));
                if (std::find(blocked.begin(), blocked.end(), key) != blocked.end()) continue;
                const uint64_t off = s->pool.alloc(c->bytes);
                if (off == UINT64_MAX) {
                    if (c->bypassed >= kMaxBypass) break;  // its turn: wait for memory
                    blocked.push_back(key);
                    continue;
                }
                c->pool_off = off;
                r = c;
                for (size_t j = 0; j < i; ++j) ++s->pending[j]->bypassed;
                s->pending.erase(s->pending.begin() + static_cast<std::ptrdiff_t>(i));
                break;
            }
            if (!r) break;  // nothing fits: wait for memory to come back
            ClientGen *g = r->type == 0 ? client_gen(s, r->client, r->kind, stream_for(s, r->client, r->kind)) : nullptr;
            s->launching.push_back(r);
            lk.unlock();  // launches can take a while (an Ising job is many kernels)
            const bool ok = (r->type != 0 || g) && launch_request(s, *r, g);
            lk.lock();
            s->launching.erase(std::find(s->launching.begin(), s->launching.end(), r));
            if (ok) {
                r->state = 1;
                s->inflight.push_back(r);
            } else {
                r->state = 3;
                r->done_at = Clock::now();
                s->completed.push_back(r->ticket);
                s->cv_done.notify_all();
            }
            progress = true;
        }
        if (!progress) {
            if (s->inflight.empty() && s->pending.empty())
                s->cv_work.wait(lk);
            else
                s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

}  // namespace

rngx_status server_create(const rngx_server_config *cfg, Server **out) {
    Server *s = new Server{};
    s->cfg = *cfg;
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess) {
        delete s;
        return hip_fail(hipErrorInvalidDevice, "device query");
    }
    if (!s->pool.init(cfg->memory_budget)) {
        delete s;
        return fail(RNGX_E_NOMEM, "cannot allocate the memory budget");
    }
    // jump tables for requests of up to kMaxServedValues values, every kind
    for (int k = RNGX_LCG32; k <= RNGX_PHILOX4X32_7; ++k) {
        const rngx_kind kind = static_cast<rngx_kind>(k);
        const uint64_t C = stream_fill_chunk(kind);
        const uint64_t steps = kind == RNGX_XS1024W ? kMaxServedValues / 32 : kMaxServedValues;
        std::vector<uint64_t> t64;
        std::vector<uint32_t> t32;
        jump_table(kind, C, (steps + C - 1) / C, &t64, &t32);
        for (int w = 0; w < 2; ++w) {
            const uint64_t bytes = w == 0 ? 8 * t64.size() : 4 * t32.size();
            if (!bytes) continue;
            const uint64_t off = s->pool.alloc(bytes);
            if (off == UINT64_MAX || hipMemcpy(s->pool.ptr(off), w == 0 ? static_cast<const void *>(t64.data())
                                                                       : static_cast<const void *>(t32.data()),
                                               bytes, hipMemcpyHostToDevice) != hipSuccess) {
                (void)hipGetLastError();
                delete s;
                return fail(RNGX_E_NOMEM, "memory budget too small for the jump tables");
            }
            if (w == 0) s->t64[k] = reinterpret_cast<const uint64_t *>(s->pool.ptr(off));
            else s->t32[k] = reinterpret_cast<const uint32_t *>(s->pool.ptr(off));
        }
    }
    for (uint32_t i = 0; i < cfg->slots; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return fail(RNGX_E_HIP, "stream creation failed");
        }
        s->streams.push_back(st);
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return RNGX_OK;
}

namespace {

rngx_status submit(Server *s, ServerRequest req, uint64_t *ticket) {
    auto r = std::make_shared<ServerRequest>(req);
    r->arrival = Clock::now();
    r->bytes = request_bytes(s, *r);
    if (r->bytes > s->pool.size())
        return fail(RNGX_E_NOMEM, "request needs " + std::to_string(r->bytes) + " bytes, more than the whole budget");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (r->type == 1) r->ising_index = s->ising_count[r->client]++;
        r->ticket = s->next_ticket++;
        s->all[r->ticket] = r;
        s->pending.push_back(r);
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return RNGX_OK;
}

}  // namespace

rngx_status server_submit_fill(Server *s, uint32_t client, rngx_kind kind, uint64_t count, int f32, uint64_t *ticket) {
    ServerRequest r{};
    r.type = 0;
    r.client = client;
    r.kind = kind;
    r.count = count;
    r.f32 = f32 ? 1 : 0;
    return submit(s, r, ticket);
}

rngx_status server_submit_ising(Server *s, uint32_t client, rngx_kind kind, uint32_t L, double beta, uint32_t sweeps,
                                uint64_t *ticket) {
    ServerRequest r{};
    r.type = 1;
    r.client = client;
    r.kind = kind;
    r.L = L;
    r.beta = beta;
    r.sweeps = sweeps;
    return submit(s, r, ticket);
}

rngx_status server_wait(Server *s, uint64_t ticket, double timeout_s, rngx_request_result *res) {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(RNGX_E_INVALID, "unknown or released ticket");
    auto r = it->second;
    const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(timeout_s));
    while (r->state < 2) {
        if (timeout_s >= 0 && s->cv_done.wait_until(lk, until) == std::cv_status::timeout && r->state < 2) {
            res->status = RNGX_E_BUSY;
            return fail(RNGX_E_BUSY, "request not finished");
        }
        if (timeout_s < 0) s->cv_done.wait(lk);
    }
    if (r->state == 3) {
        res->status = RNGX_E_HIP;
        return fail(RNGX_E_HIP, "request failed on the device");
    }
    res->status = RNGX_OK;
    res->d_output = s->pool.ptr(r->pool_off);
    res->n_values = r->n_values;
    res->latency_s = std::chrono::duration<double>(r->done_at - r->arrival).count();
    return RNGX_OK;
}

rngx_status server_wait_any(Server *s, double timeout_s, uint64_t *ticket, rngx_request_result *res) {
    std::unique_lock<std::mutex> lk(s->mu);
    const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(timeout_s));
    while (s->completed.empty()) {
        if (timeout_s < 0) {
            s->cv_done.wait(lk);
        } else if (s->cv_done.wait_until(lk, until) == std::cv_status::timeout && s->completed.empty()) {
            res->status = RNGX_E_BUSY;
            return fail(RNGX_E_BUSY, "no request finished in time");
        }
    }
    *ticket = s->completed.front();
    s->completed.pop_front();
    auto r = s->all.at(*ticket);
    if (r->state == 3) {
        res->status = RNGX_E_HIP;
        return fail(RNGX_E_HIP, "request failed on the device");
    }
    res->status = RNGX_OK;
    res->d_output = s->pool.ptr(r->pool_off);
    res->n_values = r->n_values;
    res->latency_s = std::chrono::duration<double>(r->done_at - r->arrival).count();
    return RNGX_OK;
}

rngx_status server_release(Server *s, uint64_t ticket) {
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return fail(RNGX_E_INVALID, "unknown or released ticket");
        if (it->second->state < 2) return fail(RNGX_E_BUSY, "request not finished");
        if (it->second->pool_off != UINT64_MAX) s->pool.release(it->second->pool_off);
        s->all.erase(it);
    }
    s->cv_work.notify_one();
    return RNGX_OK;
}

int server_device(const Server *s) { return s->device; }

rngx_status server_cancel(Server *s, uint64_t ticket) {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(RNGX_E_INVALID, "unknown or released ticket");
    if (it->second->state != 0) return fail(RNGX_E_BUSY, "the request was already admitted");
    for (auto p = s->pending.begin(); p != s->pending.end(); ++p)
        if ((*p)->ticket == ticket) { s->pending.erase(p); break; }
    s->all.erase(it);
    return RNGX_OK;
}

namespace {
// No request of (client, kind) pending or on the device.  Caller holds mu.
bool idle(const Server *s, uint32_t client, rngx_kind kind) {
    for (const auto &r : s->pending)
        if (r->client == client && r->kind == kind) return false;
    for (const auto &r : s->inflight)
        if (r->client == client && r->kind == kind) return false;
    for (const auto &r : s->launching)
        if (r->client == client && r->kind == kind) return false;
    return true;
}
}  // namespace

size_t server_client_state_bytes(rngx_kind kind) { return state_bytes(kind, unit_streams(kind)); }

rngx_status server_get_client_state(Server *s, uint32_t client, rngx_kind kind, void *host_buf) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!idle(s, client, kind)) return fail(RNGX_E_BUSY, "requests of this client and kind are still queued or running");
    const hipStream_t st = stream_for(s, client, kind);
    ClientGen *c = client_gen(s, client, kind, st);  // seeds it if it has not served yet
    if (!c) return fail(RNGX_E_NOMEM, "no memory for the client's generator");
    hipError_t e = hipMemcpyAsync(host_buf, c->buf[c->cur], server_client_state_bytes(kind), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "client state copy to host");
    return RNGX_OK;
}

rngx_status server_set_client_state(Server *s, uint32_t client, rngx_kind kind, const void *host_buf) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!idle(s, client, kind)) return fail(RNGX_E_BUSY, "requests of this client and kind are still queued or running");
    const hipStream_t st = stream_for(s, client, kind);
    ClientGen *c = client_gen(s, client, kind, st);
    if (!c) return fail(RNGX_E_NOMEM, "no memory for the client's generator");
    hipError_t e = hipMemcpyAsync(c->buf[c->cur], host_buf, server_client_state_bytes(kind), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "client state copy to device");
    return RNGX_OK;
}

void server_destroy(Server *s) {
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->worker.join();
    for (auto st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (auto &kv : s->gens) delete kv.second;  // their state lives in the pool
    for (auto e : s->spare_events) (void)hipEventDestroy(e);
    for (auto &kv : s->all)
        if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
    delete s;
}

}  // namespace rngx
