// Batched hashing of independent blocks of uneven size in one call.
//
// A batch plan owns (a) the twiddle tables of every transform length it has
// met, built once and reused across calls, and (b) a few worker streams, each
// with a scratch arena sized for the largest block it has run.  A call derives
// each block's plan on the host, spreads the blocks over the worker streams
// (longest first, each to the least-loaded stream), forks the workers from
// the caller's stream, enqueues every block's kernel sequence on its worker,
// and joins back.  Blocks whose transforms cannot fill the GPU alone (short
// rows, single-workgroup scan steps) then run side by side.  With graphs on,
// the fork / launches / join of a block list is captured once into a HIP
// graph and replayed by later calls with the same list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "pa_internal.hpp"

namespace {

constexpr int kLanes = 4;  // worker streams (one per hardware queue HIP gives a process by default)

struct Tables {
    uint32_t len;  // pa::len_key of the transform length
    void *base;
};

struct Lane {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    void *arena = nullptr;
    size_t bytes = 0;
};

// A captured block list: replayable while no arena or table it points into
// has been reallocated (epoch).
struct Captured {
    std::vector<pa_block> blocks;
    uint64_t epoch;
    hipGraphExec_t exec;
};
constexpr size_t kMaxGraphs = 8;

bool same_blocks(const std::vector<pa_block> &v, const pa_block *b, uint32_t count) {
    return v.size() == count && std::memcmp(v.data(), b, count * sizeof(pa_block)) == 0;
}

}  // namespace

struct pa_batch_plan {
    int device;
    uint32_t max_blocks;
    uint64_t max_total_bits;
    std::vector<Tables> tables;
    Lane lanes[kLanes];
    hipEvent_t fork;
    uint32_t *d_status;  // max_blocks words
    uint32_t *h_status;  // pinned copy
    // tuned shapes (pa_batch_plan_tune): (gamma, k) -> limb width, length
    // form and column-tile width
    std::map<std::pair<uint64_t, uint64_t>, pa_params> tuned;
    // graph replay (pa_batch_plan_set_graphs)
    bool graphs_on = false;
    hipStream_t cap = nullptr;                 // capture / replay origin stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    uint64_t epoch = 0;                        // bumped on every arena or table allocation
    std::vector<Captured> graphs;              // most recently used last
};

namespace {

void drop_graphs(pa_batch_plan *bp) {
    for (Captured &c : bp->graphs) (void)hipGraphExecDestroy(c.exec);
    bp->graphs.clear();
}

void destroy(pa_batch_plan *bp) {
    if (bp->cap) (void)hipStreamSynchronize(bp->cap);
    drop_graphs(bp);
    if (bp->cap) (void)hipStreamDestroy(bp->cap);
    if (bp->ev_in) (void)hipEventDestroy(bp->ev_in);
    if (bp->ev_out) (void)hipEventDestroy(bp->ev_out);
    for (Lane &l : bp->lanes) {
        if (l.st) (void)hipStreamSynchronize(l.st);
        if (l.arena) (void)hipFree(l.arena);
        if (l.done) (void)hipEventDestroy(l.done);
        if (l.st) (void)hipStreamDestroy(l.st);
    }
    for (Tables &t : bp->tables) (void)hipFree(t.base);
    if (bp->fork) (void)hipEventDestroy(bp->fork);
    if (bp->d_status) (void)hipFree(bp->d_status);
    if (bp->h_status) (void)hipHostFree(bp->h_status);
    (void)hipGetLastError();
    delete bp;
}

// Twiddle tables for plan p's transform length, built on `st` when new.
void *tables_for(pa_batch_plan *bp, pa_plan *p, const pa::PlanLayout &lay, hipStream_t st) {
    for (Tables &t : bp->tables)
        if (t.len == pa::len_key(*p)) return t.base;
    void *base = nullptr;
    if (hipMalloc(&base, lay.table_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    pa::bind_tables(p, base, lay);
    if (pa::launch_twiddles(p, st) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(base);
        return nullptr;
    }
    bp->tables.push_back(Tables{pa::len_key(*p), base});
    ++bp->epoch;
    return base;
}

}  // namespace

extern "C" {

pa_status pa_batch_plan_create(uint32_t max_blocks, uint64_t max_total_bits, int hip_device,
                               pa_batch_plan **out) {
    if (!out || max_blocks == 0 || max_total_bits == 0) return PA_ERR_ARG;
    *out = nullptr;
    pa::DeviceGuard guard(hip_device);
    if (!guard.ok) return PA_ERR_DEVICE;
    pa_batch_plan *bp = new (std::nothrow) pa_batch_plan();
    if (!bp) return PA_ERR_NOMEM;
    bp->device = hip_device;
    bp->max_blocks = max_blocks;
    bp->max_total_bits = max_total_bits;
    bool ok = hipEventCreateWithFlags(&bp->fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&bp->cap, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&bp->ev_in, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&bp->ev_out, hipEventDisableTiming) == hipSuccess;
    for (Lane &l : bp->lanes) {
        ok = ok && hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&l.done, hipEventDisableTiming) == hipSuccess;
    }
    ok = ok && hipMalloc((void **)&bp->d_status, (size_t)max_blocks * 4) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&bp->h_status, (size_t)max_blocks * 4, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        destroy(bp);
        return PA_ERR_NOMEM;
    }
    *out = bp;
    return PA_OK;
}

void pa_batch_plan_destroy(pa_batch_plan *bp) {
    if (!bp) return;
    pa::DeviceGuard guard(bp->device);
    destroy(bp);
}

pa_status pa_hash_batched(pa_batch_plan *bp, const pa_block *blocks, uint32_t count, pa_status *per_block,
                          hipStream_t stream) {
    if (!bp || !blocks || !per_block || count == 0) return PA_ERR_ARG;
    if (count > bp->max_blocks) return PA_ERR_LIMIT;
    uint64_t total = 0;
    for (uint32_t i = 0; i < count; ++i) total += blocks[i].n;
    if (total > bp->max_total_bits) return PA_ERR_LIMIT;
    pa::DeviceGuard guard(bp->device);
    if (!guard.ok) return PA_ERR_DEVICE;

    // host side: derive every block's plan; host-detectable errors end there
    std::vector<pa_plan> plans(count);
    std::vector<pa::PlanLayout> lays(count);
    std::vector<double> cost(count, 0.0);
    std::vector<uint32_t> order;
    for (uint32_t i = 0; i < count; ++i) {
        const pa_block &bk = blocks[i];
        pa_params prm{bk.n, bk.r, 0, 0, 0, 0, 0};
        per_block[i] = pa::derive_plan(&prm, &plans[i], &lays[i]);
        if (per_block[i] == PA_OK && !bp->tuned.empty()) {
            auto it = bp->tuned.find({plans[i].gamma, plans[i].k});
            if (it != bp->tuned.end()) {
                prm.B = it->second.B;
                prm.flags = it->second.flags;
                prm.col_lg = it->second.col_lg;
                per_block[i] = pa::derive_plan(&prm, &plans[i], &lays[i]);
            }
        }
        if (per_block[i] == PA_OK && (!bk.key || !bk.a || !bk.b || !bk.c || !bk.out)) per_block[i] = PA_ERR_ARG;
        if (per_block[i] != PA_OK) continue;
        plans[i].device = bp->device;
        cost[i] = (double)(2 * plans[i].k + 4) * (double)plans[i].N * plans[i].m;
        order.push_back(i);
    }
    if (order.empty()) return PA_OK;

    // tables for every length in the batch (built on the caller's stream)
    for (uint32_t i : order) {
        void *tb = tables_for(bp, &plans[i], lays[i], stream);
        if (!tb) return PA_ERR_NOMEM;
        pa::bind_tables(&plans[i], tb, lays[i]);
    }

    // longest first, each block to the least-loaded worker
    std::sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return cost[x] > cost[y]; });
    std::vector<uint32_t> lane_of(count, 0);
    double load[kLanes] = {};
    size_t need[kLanes] = {};
    for (uint32_t i : order) {
        int best = 0;
        for (int l = 1; l < kLanes; ++l)
            if (load[l] < load[best]) best = l;
        lane_of[i] = best;
        load[best] += cost[i];
        need[best] = std::max(need[best], lays[i].scratch_bytes);
    }
    for (int l = 0; l < kLanes; ++l) {
        Lane &ln = bp->lanes[l];
        if (need[l] <= ln.bytes) continue;
        // grow: the arena may still be in use by an earlier call on this worker
        // (or by a replayed graph, which runs outside the worker streams)
        if (ln.arena) {
            if (hipStreamSynchronize(ln.st) != hipSuccess || hipStreamSynchronize(bp->cap) != hipSuccess ||
                hipFree(ln.arena) != hipSuccess) {
                (void)hipGetLastError();
                return PA_ERR_DEVICE;
            }
            ln.arena = nullptr;
            ln.bytes = 0;
        }
        ++bp->epoch;
        if (hipMalloc(&ln.arena, need[l]) != hipSuccess) {
            (void)hipGetLastError();
            ln.arena = nullptr;
            return PA_ERR_NOMEM;
        }
        ln.bytes = need[l];
    }

    // fork from `origin`, enqueue every block on its worker, join back
    auto enqueue_all = [&](hipStream_t origin) -> pa_status {
        if (hipEventRecord(bp->fork, origin) != hipSuccess) return PA_ERR_DEVICE;
        bool used[kLanes] = {};
        for (uint32_t i : order) used[lane_of[i]] = true;
        for (int l = 0; l < kLanes; ++l)
            if (used[l] && hipStreamWaitEvent(bp->lanes[l].st, bp->fork, 0) != hipSuccess) return PA_ERR_DEVICE;
        for (uint32_t i : order) {
            const pa_block &bk = blocks[i];
            Lane &ln = bp->lanes[lane_of[i]];
            pa::bind_scratch(&plans[i], ln.arena, lays[i]);
            pa_status s = pa::enqueue_hash(&plans[i], bk.key, bk.a, bk.b, bk.c, bk.out, bp->d_status + i, nullptr,
                                           nullptr, ln.st);
            if (s != PA_OK) return s;
        }
        for (int l = 0; l < kLanes; ++l) {
            if (!used[l]) continue;
            if (hipEventRecord(bp->lanes[l].done, bp->lanes[l].st) != hipSuccess ||
                hipStreamWaitEvent(origin, bp->lanes[l].done, 0) != hipSuccess)
                return PA_ERR_DEVICE;
        }
        return PA_OK;
    };
    if (!bp->graphs_on) {
        const pa_status s = enqueue_all(stream);
        if (s != PA_OK) return s;
    } else {
        // replay the captured list, or capture it now (tables and arenas are
        // in place, so nothing below allocates); `cap` runs after `stream`'s
        // earlier work and `stream` continues after the graph
        hipGraphExec_t exec = nullptr;
        for (size_t g = 0; g < bp->graphs.size(); ++g) {
            if (bp->graphs[g].epoch == bp->epoch && same_blocks(bp->graphs[g].blocks, blocks, count)) {
                Captured c = bp->graphs[g];
                bp->graphs.erase(bp->graphs.begin() + (long)g);
                bp->graphs.push_back(c);
                exec = c.exec;
                break;
            }
        }
        if (hipEventRecord(bp->ev_in, stream) != hipSuccess || hipStreamWaitEvent(bp->cap, bp->ev_in, 0) != hipSuccess)
            return PA_ERR_DEVICE;
        if (!exec) {
            hipGraph_t graph = nullptr;
            if (hipStreamBeginCapture(bp->cap, hipStreamCaptureModeRelaxed) != hipSuccess) return PA_ERR_DEVICE;
            const pa_status s = enqueue_all(bp->cap);
            const hipError_t e = hipStreamEndCapture(bp->cap, &graph);
            if (s != PA_OK || e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                (void)hipGetLastError();
                return s != PA_OK ? s : PA_ERR_DEVICE;
            }
            const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                (void)hipGetLastError();
                return PA_ERR_DEVICE;
            }
            if (bp->graphs.size() >= kMaxGraphs) {
                // the evicted graph may still run: wait for the plan's work first
                if (hipStreamSynchronize(bp->cap) != hipSuccess) return PA_ERR_DEVICE;
                (void)hipGraphExecDestroy(bp->graphs.front().exec);
                bp->graphs.erase(bp->graphs.begin());
            }
            bp->graphs.push_back(Captured{std::vector<pa_block>(blocks, blocks + count), bp->epoch, exec});
        }
        if (hipGraphLaunch(exec, bp->cap) != hipSuccess || hipEventRecord(bp->ev_out, bp->cap) != hipSuccess ||
            hipStreamWaitEvent(stream, bp->ev_out, 0) != hipSuccess) {
            (void)hipGetLastError();
            return PA_ERR_DEVICE;
        }
    }
    if (hipMemcpyAsync(bp->h_status, bp->d_status, (size_t)count * 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipGetLastError();
        return PA_ERR_DEVICE;
    }
    for (uint32_t i : order) per_block[i] = pa_decode_status(bp->h_status[i]);
    return PA_OK;
}

pa_status pa_batch_plan_set_graphs(pa_batch_plan *bp, int enable) {
    if (!bp) return PA_ERR_ARG;
    pa::DeviceGuard guard(bp->device);
    if (!guard.ok) return PA_ERR_DEVICE;
    if (!enable) {
        if (hipStreamSynchronize(bp->cap) != hipSuccess) return PA_ERR_DEVICE;
        drop_graphs(bp);
    }
    bp->graphs_on = enable != 0;
    return PA_OK;
}

pa_status pa_batch_plan_tune(pa_batch_plan *bp, const pa_block *blocks, uint32_t count, uint32_t reps,
                             uint32_t *tuned) {
    if (tuned) *tuned = 0;
    if (!bp || (!blocks && count) || reps == 0) return PA_ERR_ARG;
    for (uint32_t i = 0; i < count; ++i) {
        pa_params prm{blocks[i].n, blocks[i].r, 0, 0, 0, 0, 0};
        pa_plan p{};
        pa::PlanLayout lay;
        if (pa::derive_plan(&prm, &p, &lay) != PA_OK) continue;
        const std::pair<uint64_t, uint64_t> key{p.gamma, p.k};
        if (bp->tuned.count(key)) continue;
        pa_params best{};
        const pa_status st = pa_plan_tune(&prm, bp->device, reps, &best, nullptr);
        if (st != PA_OK) return st;
        bp->tuned[key] = best;
        ++bp->epoch;  // captured graphs of this class's blocks are stale
        if (tuned) ++*tuned;
    }
    return PA_OK;
}

}  // extern "C"
