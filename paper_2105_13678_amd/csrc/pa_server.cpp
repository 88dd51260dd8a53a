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
// budget is exact.  The twiddle tables of each transform length and the seed
// transforms of each (session, class, shape) are resident sets in a second
// arena of the resident budget (pa_resident.hpp): shared by every slot,
// built on a stream of their own the first time a request needs them (the
// request's stream waits for the build's event, the worker does not), and
// evicted least recently used first when a new set needs room and no
// admitted request holds them.
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
#include "pa_resident.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Seeds {
    uint64_t gamma, kmax;
    uint64_t *d_a, *d_b, *d_c;  // one device allocation: kmax*W + W + W words
};

struct Request {
    uint64_t ticket = 0;
    pa_request req{};
    pa_plan plan{};  // value-initialised: no profiling, no event lists
    pa::PlanLayout lay{};
    size_t footprint = 0;  // scratch + key + output bytes on the device
    size_t offset = 0;     // placement in the arena while admitted
    pa::ResidentKey tkey{}, skey{};  // its resident sets: twiddle tables, seed transforms
    size_t tbytes = 0, sbytes = 0;
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
    void *res_arena = nullptr;        // resident_budget_bytes: twiddle tables and seed transforms
    pa::ResidentCache resident{0};
    hipStream_t build = nullptr;      // resident sets are built here
    std::vector<hipEvent_t> ev_pool;  // build events of evicted sets, for reuse
    std::vector<Slot> slots;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
};

namespace {

uint64_t seed_key(uint32_t session, uint64_t gamma) { return ((uint64_t)session << 32) ^ gamma; }

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

uint32_t shape_of(const pa_plan &p) { return p.B << 8 | pa::len_key(p); }

hipEvent_t take_event(pa_server *s) {
    if (!s->ev_pool.empty()) {
        hipEvent_t e = s->ev_pool.back();
        s->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// The resident sets of r (twiddle tables, then seed transforms): found, or
// placed (evicting idle sets) and their builds enqueued on the build stream,
// each followed by its ready event (entry->aux).  Both are held by r on
// success.  Returns false when they cannot be placed now (nothing changed
// then) or a build could not be enqueued (worker thread, lock held).
bool acquire_resident(pa_server *s, Request &r, Seeds &sd, bool *failed) {
    *failed = false;
    pa::ResidentCache &C = s->resident;
    std::vector<pa::ResidentCache::Entry> evicted;
    pa::ResidentCache::Entry *te = C.find(r.tkey);
    const bool new_t = te == nullptr;
    if (new_t) te = C.insert(r.tkey, r.tbytes, &evicted);
    if (!te) return false;
    C.acquire(te);
    pa::ResidentCache::Entry *se = C.find(r.skey);
    const bool new_s = se == nullptr;
    if (new_s) se = C.insert(r.skey, r.sbytes, &evicted);
    for (const auto &e : evicted)
        if (e.aux) s->ev_pool.push_back((hipEvent_t)e.aux);
    if (!se) {
        C.release(te);
        if (new_t) C.erase(r.tkey);
        return false;
    }
    C.acquire(se);
    char *base = (char *)s->res_arena;
    pa::bind_tables(&r.plan, base + te->off, r.lay);
    bool ok = true;
    if (new_t) {
        hipEvent_t ev = take_event(s);
        ok = ev && pa::launch_twiddles(&r.plan, s->build) == hipSuccess && hipEventRecord(ev, s->build) == hipSuccess;
        te->aux = ev;
    }
    uint32_t *d = (uint32_t *)(base + se->off);
    uint32_t *db = d + (size_t)sd.kmax * pa::NPRIMES * r.plan.N;
    if (ok && new_s) {
        hipEvent_t ev = take_event(s);
        ok = ev && pa::launch_seed_transforms(&r.plan, sd.d_a, sd.kmax, sd.d_b, d, db, s->build) == hipSuccess &&
             hipEventRecord(ev, s->build) == hipSuccess;
        se->aux = ev;
    }
    if (!ok) {
        (void)hipGetLastError();
        C.release(te);
        C.release(se);
        if (new_s) {
            if (se->aux) s->ev_pool.push_back((hipEvent_t)se->aux);
            C.erase(r.skey);
        }
        if (new_t) {
            if (te->aux) s->ev_pool.push_back((hipEvent_t)te->aux);
            C.erase(r.tkey);
        }
        *failed = true;
        return false;
    }
    r.plan.res_a = d;
    r.plan.res_b = db;
    return true;
}

void release_resident(pa_server *s, Request &r) {
    if (pa::ResidentCache::Entry *e = s->resident.find(r.tkey)) s->resident.release(e);
    if (pa::ResidentCache::Entry *e = s->resident.find(r.skey)) s->resident.release(e);
}

// Enqueue request r on slot sl (worker thread), its resident sets acquired:
// the slot's stream waits for their builds.  Returns PA_OK or an error (then
// nothing of r is in flight).
pa_status launch(pa_server *s, Slot &sl, Request &r, Seeds &sd, hipEvent_t ev_t, hipEvent_t ev_s) {
    char *base = (char *)s->arena + r.offset;
    pa::bind_scratch(&r.plan, base, r.lay);
    uint64_t *d_key = (uint64_t *)(base + r.lay.scratch_bytes);
    uint64_t *d_out = (uint64_t *)(base + r.lay.scratch_bytes + align256(r.plan.key_words * 8));
    const size_t key_bytes = (size_t)r.plan.key_words * 8, out_bytes = (size_t)r.plan.out_words * 8;
    if (hipEventRecord(sl.ev0, sl.st) != hipSuccess ||
        hipMemcpyAsync(d_key, r.req.key, key_bytes, hipMemcpyHostToDevice, sl.st) != hipSuccess ||
        hipStreamWaitEvent(sl.st, ev_t, 0) != hipSuccess || hipStreamWaitEvent(sl.st, ev_s, 0) != hipSuccess) {
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
            release_resident(s, sl.cur);
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
            // presence checked at submission; seeds are never removed, and map
            // nodes stay put, so the reference outlives the lock
            Seeds &sd = s->seeds.find(seed_key(head.req.session, head.plan.gamma))->second;
            bool failed = false;
            if (!acquire_resident(s, head, sd, &failed) && !failed) {
                s->placer.release(off);  // the resident sets in use leave no room yet
                break;
            }
            Request r = head;
            r.offset = off;
            s->queue.pop_front();
            r.t_admit = Clock::now();
            if (failed) {
                s->placer.release(off);
                lk.unlock();
                finish(s, r, PA_ERR_DEVICE, 0.0);
                lk.lock();
                continue;
            }
            const hipEvent_t ev_t = (hipEvent_t)s->resident.find(r.tkey)->aux;
            const hipEvent_t ev_s = (hipEvent_t)s->resident.find(r.skey)->aux;
            free_slot->busy = true;
            free_slot->cur = r;
            lk.unlock();
            pa_status e = launch(s, *free_slot, free_slot->cur, sd, ev_t, ev_s);
            lk.lock();
            if (e != PA_OK) {
                free_slot->busy = false;
                s->placer.release(r.offset);
                release_resident(s, r);
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
    if (s->build) (void)hipStreamSynchronize(s->build);
    for (const auto &e : s->resident.all())
        if (e.aux) (void)hipEventDestroy((hipEvent_t)e.aux);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    if (s->build) (void)hipStreamDestroy(s->build);
    for (auto &kv : s->seeds) (void)hipFree(kv.second.d_a);
    if (s->arena) (void)hipFree(s->arena);
    if (s->res_arena) (void)hipFree(s->res_arena);
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
    if (s->cfg.resident_budget_bytes == 0) s->cfg.resident_budget_bytes = cfg->hbm_budget_bytes;
    if (hipMalloc(&s->arena, cfg->hbm_budget_bytes) != hipSuccess ||
        hipMalloc(&s->res_arena, s->cfg.resident_budget_bytes) != hipSuccess ||
        hipStreamCreateWithFlags(&s->build, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        release(s);
        return PA_ERR_NOMEM;
    }
    s->placer.size = cfg->hbm_budget_bytes;
    s->resident = pa::ResidentCache(s->cfg.resident_budget_bytes);
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
    r.tkey = pa::ResidentKey{0, 0, 0, shape_of(r.plan)};
    r.skey = pa::ResidentKey{1, req->session, r.plan.gamma, shape_of(r.plan)};
    r.tbytes = r.lay.table_bytes;
    r.t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->seeds.find(seed_key(req->session, r.plan.gamma));
        if (it == s->seeds.end() || it->second.kmax < r.plan.k) return PA_ERR_ARG;
        // the seed transforms: kmax + 1 arrays of 3 x N words; with the
        // tables they must fit the resident budget on their own
        r.sbytes = (size_t)(it->second.kmax + 1) * pa::NPRIMES * r.plan.N * 4;
        if (align256(r.tbytes) + align256(r.sbytes) > s->cfg.resident_budget_bytes) return PA_ERR_LIMIT;
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
