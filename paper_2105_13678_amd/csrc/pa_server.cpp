// Serving loop: requests from many QKD sessions hashed as they arrive.
//
// pa_submit queues a request (host key in, host output out) and returns a
// ticket at once; a worker thread admits queued requests in arrival order
// while a worker slot and the device-memory budget allow, and runs each one
// on its slot's stream: key upload, the hash (with the session's seeds and
// their transforms, which stay resident on the device, so a request costs
// k + 3 transforms instead of 2k + 4), output and status download,
// completion event.  pa_poll reports PA_PENDING until the request is done, then its
// status and timing.  Each admitted request's device memory (scratch, key,
// output) is placed first-fit in one arena of the configured budget, so the
// budget is exact.  Twiddle tables are built once per transform length and
// shared by every slot.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <new>
#include <thread>
#include <vector>

#include "pa_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Seeds {
    uint64_t gamma, kmax;
    uint64_t *d_a, *d_b, *d_c;  // one device allocation: kmax*W + W + W words
    // column-pass transforms of a (kmax x 3 x N words) and b (3 x N words),
    // per transform shape (limb width B << 8 | pa::len_key), built on first use
    std::map<uint32_t, uint32_t *> trans;
};

struct Request {
    uint64_t ticket = 0;
    pa_request req{};
    pa_plan plan{};  // value-initialised: no profiling, no event lists
    pa::PlanLayout lay{};
    size_t footprint = 0;  // scratch + key + output bytes on the device
    size_t offset = 0;     // placement in the arena while admitted
    Clock::time_point t_submit, t_admit;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    uint32_t *h_status = nullptr;  // pinned word
    bool busy = false;
    Request cur;
};

// First-fit placement of byte ranges in [0, size), 256-byte aligned.
struct Placer {
    size_t size = 0;
    std::map<size_t, size_t> used;  // offset -> bytes
    bool place(size_t bytes, size_t *off) {
        size_t start = 0;
        for (const auto &u : used) {
            if (u.first >= start && u.first - start >= bytes) break;
            start = align256(u.first + u.second);
        }
        if (start > size || size - start < bytes) return false;
        used[start] = bytes;
        *off = start;
        return true;
    }
    void release(size_t off) { used.erase(off); }
};

struct Done {
    pa_status status;
    pa_timing timing;
};

}  // namespace

struct pa_server {
    pa_server_cfg cfg;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> queue;
    std::set<uint64_t> pending;  // queued or running
    std::map<uint64_t, Done> done;
    void *arena = nullptr;       // hbm_budget_bytes
    Placer placer;
    std::map<uint64_t, Seeds> seeds;  // key: seed_key(session, gamma)
    std::vector<std::pair<uint32_t, void *>> tables;  // transform length -> twiddle tables
    std::vector<Slot> slots;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
};

namespace {

uint64_t seed_key(uint32_t session, uint64_t gamma) { return ((uint64_t)session << 32) ^ gamma; }

// Twiddle tables for r's transform length; built synchronously on `st` the
// first time (worker thread only).
void *tables_for(pa_server *s, Request &r, hipStream_t st) {
    for (auto &t : s->tables)
        if (t.first == pa::len_key(r.plan)) return t.second;
    void *base = nullptr;
    if (hipMalloc(&base, r.lay.table_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    pa::bind_tables(&r.plan, base, r.lay);
    if (pa::launch_twiddles(&r.plan, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(base);
        return nullptr;
    }
    s->tables.emplace_back(pa::len_key(r.plan), base);
    return base;
}

void finish(pa_server *s, Request &r, pa_status st, double device_ms) {
    Done d;
    d.status = st;
    d.timing.queued_ms = ms_between(r.t_submit, r.t_admit);
    d.timing.device_ms = device_ms;
    d.timing.total_ms = ms_between(r.t_submit, Clock::now());
    std::lock_guard<std::mutex> g(s->mu);
    s->pending.erase(r.ticket);
    s->done[r.ticket] = d;
}

// Resident seed transforms of sd for r's shape; built synchronously on `st`
// the first time (worker thread only).
uint32_t *seed_transforms(Seeds &sd, Request &r, hipStream_t st) {
    const uint32_t key = r.plan.B << 8 | pa::len_key(r.plan);
    auto it = sd.trans.find(key);
    if (it != sd.trans.end()) return it->second;
    const size_t words = (size_t)(sd.kmax + 1) * pa::NPRIMES * r.plan.N;
    uint32_t *d = nullptr;
    if (hipMalloc((void **)&d, words * 4) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    uint32_t *db = d + (size_t)sd.kmax * pa::NPRIMES * r.plan.N;
    if (pa::launch_seed_transforms(&r.plan, sd.d_a, sd.kmax, sd.d_b, d, db, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(d);
        return nullptr;
    }
    sd.trans[key] = d;
    return d;
}

// Enqueue request r on slot sl (worker thread).  Returns PA_OK or an error
// (then nothing of r is in flight).
pa_status launch(pa_server *s, Slot &sl, Request &r, Seeds &sd) {
    // r's arena range: scratch, then the key, then the output
    void *tb = tables_for(s, r, sl.st);
    if (!tb) return PA_ERR_NOMEM;
    pa::bind_tables(&r.plan, tb, r.lay);
    uint32_t *tr = seed_transforms(sd, r, sl.st);
    if (!tr) return PA_ERR_NOMEM;
    r.plan.res_a = tr;
    r.plan.res_b = tr + (size_t)sd.kmax * pa::NPRIMES * r.plan.N;
    char *base = (char *)s->arena + r.offset;
    pa::bind_scratch(&r.plan, base, r.lay);
    uint64_t *d_key = (uint64_t *)(base + r.lay.scratch_bytes);
    uint64_t *d_out = (uint64_t *)(base + r.lay.scratch_bytes + align256(r.plan.key_words * 8));
    const size_t key_bytes = (size_t)r.plan.key_words * 8, out_bytes = (size_t)r.plan.out_words * 8;
    if (hipEventRecord(sl.ev0, sl.st) != hipSuccess ||
        hipMemcpyAsync(d_key, r.req.key, key_bytes, hipMemcpyHostToDevice, sl.st) != hipSuccess) {
        (void)hipGetLastError();
        return PA_ERR_DEVICE;
    }
    pa_status e = pa::enqueue_hash(&r.plan, d_key, sd.d_a, sd.d_b, sd.d_c, d_out, r.plan.status_out, nullptr,
                                   nullptr, sl.st);
    if (e != PA_OK) return e;
    if (hipMemcpyAsync(r.req.out, d_out, out_bytes, hipMemcpyDeviceToHost, sl.st) != hipSuccess ||
        hipMemcpyAsync(sl.h_status, r.plan.status_out, 4, hipMemcpyDeviceToHost, sl.st) != hipSuccess ||
        hipEventRecord(sl.ev1, sl.st) != hipSuccess) {
        (void)hipGetLastError();
        return PA_ERR_DEVICE;
    }
    return PA_OK;
}

void worker_main(pa_server *s) {
    (void)hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // retire finished requests
        bool any_busy = false;
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.ev1);
            if (q == hipErrorNotReady) {
                any_busy = true;
                continue;
            }
            float dev_ms = 0.f;
            pa_status st;
            if (q == hipSuccess && hipEventElapsedTime(&dev_ms, sl.ev0, sl.ev1) == hipSuccess) {
                st = pa_decode_status(*sl.h_status);
            } else {
                (void)hipGetLastError();
                st = PA_ERR_DEVICE;
            }
            sl.busy = false;
            s->placer.release(sl.cur.offset);
            Request r = sl.cur;
            lk.unlock();
            finish(s, r, st, dev_ms);
            lk.lock();
        }
        // admit in arrival order while a slot and the budget allow
        while (!s->queue.empty()) {
            Request &head = s->queue.front();
            Slot *free_slot = nullptr;
            for (Slot &sl : s->slots)
                if (!sl.busy) {
                    free_slot = &sl;
                    break;
                }
            size_t off = 0;
            if (!free_slot || !s->placer.place(head.footprint, &off)) break;
            Request r = head;
            r.offset = off;
            s->queue.pop_front();
            // presence checked at submission; seeds are never removed, and map
            // nodes stay put, so the reference outlives the lock
            Seeds &sd = s->seeds.find(seed_key(r.req.session, r.plan.gamma))->second;
            r.t_admit = Clock::now();
            free_slot->busy = true;
            free_slot->cur = r;
            lk.unlock();
            pa_status e = launch(s, *free_slot, free_slot->cur, sd);
            lk.lock();
            if (e != PA_OK) {
                free_slot->busy = false;
                s->placer.release(r.offset);
                lk.unlock();
                finish(s, r, e, 0.0);
                lk.lock();
            } else {
                any_busy = true;
            }
        }
        if (s->stop && s->queue.empty() && !any_busy) break;
        if (any_busy) {
            // completions are polled: short waits keep the latency low
            s->cv.wait_for(lk, std::chrono::microseconds(50));
        } else {
            s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
        }
    }
}

void release(pa_server *s) {
    for (Slot &sl : s->slots) {
        if (sl.st) (void)hipStreamSynchronize(sl.st);
        if (sl.ev0) (void)hipEventDestroy(sl.ev0);
        if (sl.ev1) (void)hipEventDestroy(sl.ev1);
        if (sl.h_status) (void)hipHostFree(sl.h_status);
        if (sl.st) (void)hipStreamDestroy(sl.st);
    }
    for (auto &t : s->tables) (void)hipFree(t.second);
    for (auto &kv : s->seeds) {
        (void)hipFree(kv.second.d_a);
        for (auto &t : kv.second.trans) (void)hipFree(t.second);
    }
    if (s->arena) (void)hipFree(s->arena);
    (void)hipGetLastError();
    delete s;
}

}  // namespace

extern "C" {

pa_status pa_server_create(const pa_server_cfg *cfg, pa_server **out) {
    if (!cfg || !out || cfg->max_inflight == 0 || cfg->max_inflight > 64 || cfg->hbm_budget_bytes == 0)
        return PA_ERR_ARG;
    *out = nullptr;
    pa::DeviceGuard guard(cfg->device);
    if (!guard.ok) return PA_ERR_DEVICE;
    pa_server *s = new (std::nothrow) pa_server();
    if (!s) return PA_ERR_NOMEM;
    s->cfg = *cfg;
    if (hipMalloc(&s->arena, cfg->hbm_budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        s->arena = nullptr;
        release(s);
        return PA_ERR_NOMEM;
    }
    s->placer.size = cfg->hbm_budget_bytes;
    s->slots.resize(cfg->max_inflight);
    for (Slot &sl : s->slots) {
        bool ok = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreate(&sl.ev0) == hipSuccess && hipEventCreate(&sl.ev1) == hipSuccess &&
                  hipHostMalloc((void **)&sl.h_status, 64, hipHostMallocDefault) == hipSuccess;
        if (!ok) {
            release(s);
            return PA_ERR_NOMEM;
        }
    }
    try {
        s->worker = std::thread(worker_main, s);
    } catch (...) {
        release(s);
        return PA_ERR_NOMEM;
    }
    *out = s;
    return PA_OK;
}

void pa_server_destroy(pa_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    pa::DeviceGuard guard(s->cfg.device);
    release(s);
}

pa_status pa_server_set_seeds(pa_server *s, uint32_t session, uint64_t gamma, uint64_t kmax, const uint64_t *a,
                              const uint64_t *b, const uint64_t *c) {
    if (!s || !a || !b || !c || kmax == 0 || kmax > 4096) return PA_ERR_ARG;
    // gamma must be a tabled Mersenne exponent: ask the plan rule with r = 1
    pa_params prm{gamma + 1, 1, gamma, 0, 0, 0, 0};
    pa_plan tmp{};
    pa::PlanLayout lay;
    pa_status st = pa::derive_plan(&prm, &tmp, &lay);
    if (st != PA_OK && st != PA_ERR_INEXACT && st != PA_ERR_LIMIT) return st;
    const uint64_t W = (gamma + 63) / 64;
    pa::DeviceGuard guard(s->cfg.device);
    if (!guard.ok) return PA_ERR_DEVICE;
    const size_t words = (size_t)(kmax + 2) * W;
    uint64_t *d = nullptr;
    if (hipMalloc((void **)&d, words * 8) != hipSuccess) {
        (void)hipGetLastError();
        return PA_ERR_NOMEM;
    }
    if (hipMemcpy(d, a, (size_t)kmax * W * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d + kmax * W, b, W * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d + (kmax + 1) * W, c, W * 8, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(d);
        return PA_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> g(s->mu);
    const uint64_t key = seed_key(session, gamma);
    if (s->seeds.count(key)) {  // resident seeds are never replaced (requests may be using them)
        (void)hipFree(d);
        return PA_ERR_BUSY;
    }
    Seeds &sd = s->seeds[key];
    sd.gamma = gamma;
    sd.kmax = kmax;
    sd.d_a = d;
    sd.d_b = d + kmax * W;
    sd.d_c = d + (kmax + 1) * W;
    return PA_OK;
}

pa_status pa_submit(pa_server *s, const pa_request *req, uint64_t *ticket) {
    if (!s || !req || !ticket || !req->key || !req->out) return PA_ERR_ARG;
    Request r{};
    r.req = *req;
    pa_params prm{req->n, req->r, 0, 0, 0, 0, 0};
    pa_status st = pa::derive_plan(&prm, &r.plan, &r.lay);
    if (st != PA_OK) return st;
    r.plan.device = s->cfg.device;
    r.footprint = r.lay.scratch_bytes + align256(r.plan.key_words * 8) + align256(r.plan.out_words * 8);
    if (r.footprint > s->cfg.hbm_budget_bytes) return PA_ERR_LIMIT;
    r.t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->seeds.find(seed_key(req->session, r.plan.gamma));
        if (it == s->seeds.end() || it->second.kmax < r.plan.k) return PA_ERR_ARG;
        if (s->stop) return PA_ERR_BUSY;
        r.ticket = s->next_ticket++;
        *ticket = r.ticket;
        s->pending.insert(r.ticket);
        s->queue.push_back(r);
    }
    s->cv.notify_all();
    return PA_OK;
}

pa_status pa_poll(pa_server *s, uint64_t ticket, pa_status *result, pa_timing *timing) {
    if (!s || !result) return PA_ERR_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->done.find(ticket);
    if (it == s->done.end()) return s->pending.count(ticket) ? PA_PENDING : PA_ERR_ARG;
    *result = it->second.status;
    if (timing) *timing = it->second.timing;
    s->done.erase(it);
    return PA_OK;
}

}  // extern "C"
