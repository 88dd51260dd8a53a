// Batched hashing of independent blocks of uneven size in one call.
//
// A call derives each block's plan on the host and records each block's
// kernel launches (the same sequence pa_hash runs, each launch tagged with
// its step) instead of launching them.  Every step is then run for all
// blocks at once: the launches of one step that use the same kernel instance
// (same workgroup size and dynamic LDS) become one multi-block launch, whose
// workgroups find their block and their position in that block's grid in a
// small table (block placement, owner of each 8 workgroups, the blocks'
// argument structs) uploaded once per call.  A 64-block call then issues a
// few dozen launches instead of about a thousand, and blocks too small to
// fill the GPU alone share each launch with the others.  Each block has its
// own scratch in one arena (all blocks are in flight together); the twiddle
// tables of every transform length met are built once and kept.  With graphs
// on, the launches of a block list are captured once into a HIP graph (its
// tables in a device buffer of its own) and replayed by later calls with the
// same list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "pa_internal.hpp"
#include "pa_multi.hpp"

namespace {

struct Tables {
    uint32_t len;  // pa::len_key of the transform length
    void *base;
};

// One launch of a step: a multi-block launch over `members` (indices into
// the call's recorded launches), or a plain launch when there is one member.
struct Group {
    const void *single, *multi;
    dim3 block;
    uint32_t lds;
    uint32_t args_size;
    std::vector<const pa::KLaunch *> members;
    uint32_t total;                      // workgroups of the multi launch
    size_t o_args, o_geo, o_owner, end;  // table offsets
};

// A captured block list: replayable while no arena or table it points into
// has been reallocated (epoch).
struct Captured {
    std::vector<pa_block> blocks;
    uint64_t epoch;
    hipGraphExec_t exec;
    void *d_tab;  // the list's launch tables
};
constexpr size_t kMaxGraphs = 8;

bool same_blocks(const std::vector<pa_block> &v, const pa_block *b, uint32_t count) {
    return v.size() == count && std::memcmp(v.data(), b, count * sizeof(pa_block)) == 0;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// With PA_DEBUG set in the environment, device errors of a batched call are
// reported on stderr (the HIP error and the source line).
pa_status device_error(int line) {
    static const bool on = std::getenv("PA_DEBUG") != nullptr;
    const hipError_t e = hipGetLastError();
    if (on) std::fprintf(stderr, "pa_hash_batched: device error at pa_batch.cpp:%d: %s\n", line, hipGetErrorString(e));
    return PA_ERR_DEVICE;
}
#define PA_DEVICE_ERROR device_error(__LINE__)

}  // namespace

struct pa_batch_plan {
    int device;
    uint32_t max_blocks;
    uint64_t max_total_bits;
    std::vector<Tables> tables;
    void *arena = nullptr;     // every block's scratch, side by side
    size_t arena_bytes = 0;
    void *d_tab = nullptr;     // launch tables of the current call
    size_t d_tab_bytes = 0;
    unsigned char *h_tab = nullptr;  // pinned staging of the launch tables
    size_t h_tab_bytes = 0;
    uint32_t *d_status;  // max_blocks words
    uint32_t *h_status;  // pinned copy
    // tuned shapes (pa_batch_plan_tune): (gamma, k) -> limb width, length
    // form and column-tile width
    std::map<std::pair<uint64_t, uint64_t>, pa_params> tuned;
    // graph replay (pa_batch_plan_set_graphs)
    bool graphs_on = false;
    hipStream_t cap = nullptr;                 // capture / replay origin stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // a second stream for the independent launches of one step (see launch_groups)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    uint64_t epoch = 0;                        // bumped on every arena or table allocation
    std::vector<Captured> graphs;              // most recently used last
};

namespace {

void drop_graphs(pa_batch_plan *bp) {
    for (Captured &c : bp->graphs) {
        (void)hipGraphExecDestroy(c.exec);
        (void)hipFree(c.d_tab);
    }
    bp->graphs.clear();
}

void destroy(pa_batch_plan *bp) {
    if (bp->cap) (void)hipStreamSynchronize(bp->cap);
    (void)hipDeviceSynchronize();
    drop_graphs(bp);
    if (bp->cap) (void)hipStreamDestroy(bp->cap);
    if (bp->side) (void)hipStreamDestroy(bp->side);
    if (bp->ev_in) (void)hipEventDestroy(bp->ev_in);
    if (bp->ev_out) (void)hipEventDestroy(bp->ev_out);
    if (bp->ev_fork) (void)hipEventDestroy(bp->ev_fork);
    if (bp->ev_join) (void)hipEventDestroy(bp->ev_join);
    if (bp->arena) (void)hipFree(bp->arena);
    if (bp->d_tab) (void)hipFree(bp->d_tab);
    if (bp->h_tab) (void)hipHostFree(bp->h_tab);
    for (Tables &t : bp->tables) (void)hipFree(t.base);
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

std::vector<pa::MultiMember> members_of(const Group &g) {
    std::vector<pa::MultiMember> v;
    for (const pa::KLaunch *L : g.members) v.push_back(pa::MultiMember{L->grid.x, L->grid.y, L->grid.z, L->args});
    return v;
}

// Group the recorded launches step by step (same kernel instance, workgroup
// size and LDS: one launch) and lay out the tables of each multi-block
// launch (pa_multi.hpp).  Returns the table bytes.
size_t build_groups(const std::vector<std::vector<pa::KLaunch>> &recs, const std::vector<uint32_t> &order,
                    std::vector<Group> &groups, size_t off0 = 0) {
    size_t off = off0;
    for (int step = 0; step < pa::SP_COUNT; ++step) {
        const size_t first = groups.size();
        for (uint32_t i : order)
            for (const pa::KLaunch &L : recs[i]) {
                if (L.step != step) continue;
                Group *g = nullptr;
                for (size_t j = first; j < groups.size(); ++j)
                    if (groups[j].single == L.single && groups[j].lds == L.lds && groups[j].block.x == L.block.x &&
                        groups[j].block.y == L.block.y && groups[j].block.z == L.block.z)
                        g = &groups[j];
                if (!g) {
                    groups.push_back(Group{L.single, L.multi, L.block, L.lds, L.args_size, {}, 0, 0, 0, 0, 0});
                    g = &groups.back();
                }
                g->members.push_back(&L);
            }
        for (size_t j = first; j < groups.size(); ++j) {
            Group &g = groups[j];
            if (g.members.size() == 1) continue;  // a plain launch
            const pa::MultiLayout lay = pa::multi_layout(members_of(g), g.args_size, off);
            g.total = lay.total;
            g.o_args = lay.o_args;
            g.o_geo = lay.o_geo;
            g.o_owner = lay.o_owner;
            g.end = lay.end;
            off = lay.end;
        }
    }
    return off;
}

// Tables of groups [g0, g1) into the staging buffer `h`; returns their byte
// range [*lo, *hi) (empty when every group is a plain launch).
void fill_tables(const std::vector<Group> &groups, size_t g0, size_t g1, unsigned char *h, size_t *lo, size_t *hi) {
    *lo = *hi = 0;
    for (size_t gi = g0; gi < g1; ++gi) {
        const Group &g = groups[gi];
        if (g.members.size() == 1) continue;
        if (*hi == 0) *lo = g.o_args;
        *hi = g.end;
        const std::vector<pa::MultiMember> mem = members_of(g);
        const pa::MultiLayout lay = pa::multi_layout(mem, g.args_size, g.o_args);
        pa::multi_fill(mem, g.args_size, lay, h);
    }
}

// End of the run of groups that starts at g0 and belongs to one step.
size_t step_end(const std::vector<Group> &groups, size_t g0) {
    size_t g1 = g0;
    while (g1 < groups.size() && groups[g1].members[0]->step == groups[g0].members[0]->step) ++g1;
    return g1;
}

hipError_t launch_one(const Group &g, const unsigned char *d_tab, hipStream_t st) {
    if (g.members.size() == 1) {
        const pa::KLaunch &L = *g.members[0];
        void *args[] = {(void *)L.args};
        return hipLaunchKernel(g.single, L.grid, g.block, args, g.lds, st);
    }
    const void *tab = d_tab + g.o_args, *geo = d_tab + g.o_geo, *owner = d_tab + g.o_owner;
    void *args[] = {(void *)&tab, (void *)&geo, (void *)&owner};
    return hipLaunchKernel(g.multi, dim3(g.total), g.block, args, g.lds, st);
}

// Threads a group launches (its work estimate).
double group_threads(const Group &g) {
    const double wg = g.members.size() == 1
                          ? (double)g.members[0]->grid.x * g.members[0]->grid.y * g.members[0]->grid.z
                          : (double)g.total;
    return wg * g.block.x * g.block.y * g.block.z;
}

// Launch groups [g0, g1) on st, step by step.  The launches of one step use
// different kernel instances for different blocks and are independent, so
// with bp (graph capture) a step's groups are split over st and the plan's
// side stream (largest first, each to the stream with less work so far),
// after an event fork and before an event join: the captured graph then
// holds them as parallel branches, and a small or latency-bound instance
// overlaps the others (64 small blocks: 0.79 -> 0.70 ms per replay).  Issued
// directly, the fork and join events cost more than the overlap gains (the
// 64 uneven blocks 10.1 -> 10.3 ms), so direct calls pass no bp.
hipError_t launch_groups(const std::vector<Group> &groups, size_t g0, size_t g1, const unsigned char *d_tab,
                         hipStream_t st, const pa_batch_plan *bp) {
    static const bool dbg = std::getenv("PA_DEBUG") != nullptr;
    for (size_t s0 = g0; s0 < g1;) {
        const size_t s1 = std::min(step_end(groups, s0), g1);
        const bool split = bp && bp->side && s1 - s0 > 1;
        if (split && (hipEventRecord(bp->ev_fork, st) != hipSuccess ||
                      hipStreamWaitEvent(bp->side, bp->ev_fork, 0) != hipSuccess))
            return hipErrorUnknown;
        std::vector<size_t> idx;
        for (size_t gi = s0; gi < s1; ++gi) idx.push_back(gi);
        if (split)
            std::stable_sort(idx.begin(), idx.end(),
                             [&](size_t a, size_t b) { return group_threads(groups[a]) > group_threads(groups[b]); });
        double w_main = 0, w_side = 0;
        for (size_t gi : idx) {
            const Group &g = groups[gi];
            const bool to_side = split && w_side < w_main;
            (to_side ? w_side : w_main) += group_threads(g);
            const hipError_t e = launch_one(g, d_tab, to_side ? bp->side : st);
            if (e != hipSuccess) {
                if (dbg)
                    std::fprintf(stderr, "pa_hash_batched: launch %zu (step %d, %zu blocks, %u workgroups of %u, lds %u): %s\n",
                                 gi, g.members[0]->step, g.members.size(), g.members.size() == 1 ? 0u : g.total,
                                 g.block.x * g.block.y * g.block.z, g.lds, hipGetErrorString(e));
                return e;
            }
        }
        if (split && (hipEventRecord(bp->ev_join, bp->side) != hipSuccess ||
                      hipStreamWaitEvent(st, bp->ev_join, 0) != hipSuccess))
            return hipErrorUnknown;
        s0 = s1;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

pa_status pa_batch_plan_create(uint32_t max_blocks, uint64_t max_total_bits, int hip_device,
                               pa_batch_plan **out) {
    if (!out || max_blocks == 0 || max_total_bits == 0) return PA_ERR_ARG;
    if (max_blocks > 65535) return PA_ERR_LIMIT;  // owner tables hold 16-bit block indices
    *out = nullptr;
    pa::DeviceGuard guard(hip_device);
    if (!guard.ok) return PA_ERR_DEVICE;
    pa_batch_plan *bp = new (std::nothrow) pa_batch_plan();
    if (!bp) return PA_ERR_NOMEM;
    bp->device = hip_device;
    bp->max_blocks = max_blocks;
    bp->max_total_bits = max_total_bits;
    bool ok = hipStreamCreateWithFlags(&bp->cap, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&bp->ev_in, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&bp->ev_out, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&bp->side, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&bp->ev_fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&bp->ev_join, hipEventDisableTiming) == hipSuccess;
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
    if (!guard.ok) return PA_DEVICE_ERROR;

    // host side: derive every block's plan; host-detectable errors end there
    std::vector<pa_plan> plans(count);
    std::vector<pa::PlanLayout> lays(count);
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
        order.push_back(i);
    }
    if (order.empty()) return PA_OK;

    // tables for every length in the batch (built on the caller's stream)
    for (uint32_t i : order) {
        void *tb = tables_for(bp, &plans[i], lays[i], stream);
        if (!tb) return PA_ERR_NOMEM;
        pa::bind_tables(&plans[i], tb, lays[i]);
    }

    // one scratch region per block, side by side in the arena
    std::vector<size_t> at(count, 0);
    size_t need = 0;
    for (uint32_t i : order) {
        at[i] = need;
        need = align_up(need + lays[i].scratch_bytes, 256);
    }
    if (need > bp->arena_bytes) {
        // the arena may still be in use by a replayed graph of an earlier call
        if (bp->arena && (hipStreamSynchronize(bp->cap) != hipSuccess || hipFree(bp->arena) != hipSuccess)) {
            (void)hipGetLastError();
            return PA_DEVICE_ERROR;
        }
        bp->arena = nullptr;
        bp->arena_bytes = 0;
        ++bp->epoch;
        if (hipMalloc(&bp->arena, need) != hipSuccess) {
            (void)hipGetLastError();
            bp->arena = nullptr;
            return PA_ERR_NOMEM;
        }
        bp->arena_bytes = need;
    }

    // record every block's launches, then group them step by step
    std::vector<std::vector<pa::KLaunch>> recs(count);
    for (uint32_t i : order) {
        const pa_block &bk = blocks[i];
        pa::bind_scratch(&plans[i], (char *)bp->arena + at[i], lays[i]);
        recs[i].reserve(24);
        plans[i].rec = &recs[i];
        const pa_status s = pa::enqueue_hash(&plans[i], bk.key, bk.a, bk.b, bk.c, bk.out, bp->d_status + i, nullptr,
                                             nullptr, stream);
        plans[i].rec = nullptr;
        if (s != PA_OK) return s == PA_ERR_DEVICE ? PA_DEVICE_ERROR : s;
    }
    // Direct launches of a small batch (below kTwoStreamBits key bits, where
    // the launches, not the GPU's arithmetic, set the time): the blocks in two
    // halves of about equal size, each run step by step on its own stream (the
    // caller's and the plan's side stream), joined at the end, so that the
    // halves' launches overlap; only the start and the end cross streams.
    // 64 blocks of 2^14 - 2^18 bits: 0.87 -> 0.78 ms per call; 64 blocks of
    // 2^22 - 2^28 bits (GPU-bound): 10.0 -> 10.2 ms, so large batches keep one
    // stream.  Graph capture: one list (its steps are split in the capture).
    constexpr uint64_t kTwoStreamBits = 1ull << 27;
    std::vector<Group> groups, groups2;
    size_t tab_bytes;
    if (!bp->graphs_on && order.size() >= 2 && total < kTwoStreamBits) {
        std::vector<uint32_t> by_size(order);
        std::stable_sort(by_size.begin(), by_size.end(),
                         [&](uint32_t x, uint32_t y) { return blocks[x].n > blocks[y].n; });
        std::vector<uint32_t> half[2];
        uint64_t load[2] = {0, 0};
        for (uint32_t i : by_size) {
            const int h = load[1] < load[0] ? 1 : 0;
            half[h].push_back(i);
            load[h] += blocks[i].n;
        }
        std::sort(half[0].begin(), half[0].end());
        std::sort(half[1].begin(), half[1].end());
        const size_t end0 = build_groups(recs, half[0], groups, 0);
        tab_bytes = build_groups(recs, half[1], groups2, end0);
    } else {
        tab_bytes = build_groups(recs, order, groups, 0);
    }
    auto grow = [](void **buf, size_t *have, size_t want, bool host) -> bool {
        if (want <= *have) return true;
        if (*buf) (void)(host ? hipHostFree(*buf) : hipFree(*buf));
        *buf = nullptr;
        *have = 0;
        const size_t sz = align_up(want + want / 2, 4096);
        const hipError_t e = host ? hipHostMalloc(buf, sz, hipHostMallocDefault) : hipMalloc(buf, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *buf = nullptr;
            return false;
        }
        *have = sz;
        return true;
    };
    // the staging buffer and the device tables are free: the previous call synchronised
    if (tab_bytes && !grow((void **)&bp->h_tab, &bp->h_tab_bytes, tab_bytes, true)) return PA_ERR_NOMEM;

    if (!bp->graphs_on) {
        if (tab_bytes && !grow(&bp->d_tab, &bp->d_tab_bytes, tab_bytes, false)) return PA_ERR_NOMEM;
        // step by step: stage and upload one step's tables, then launch the
        // step, so the device starts on the first steps while the host still
        // prepares the later ones (each step's table range is its own); each
        // half uploads its tables on its own stream
        const bool two = !groups2.empty();
        if (two && (hipEventRecord(bp->ev_fork, stream) != hipSuccess ||
                    hipStreamWaitEvent(bp->side, bp->ev_fork, 0) != hipSuccess)) {
            (void)hipGetLastError();
            return PA_DEVICE_ERROR;
        }
        auto run_step = [&](const std::vector<Group> &gs, size_t g0, hipStream_t st) -> size_t {
            const size_t g1 = step_end(gs, g0);
            size_t lo, hi;
            fill_tables(gs, g0, g1, bp->h_tab, &lo, &hi);
            if (hi > lo && hipMemcpyAsync((unsigned char *)bp->d_tab + lo, bp->h_tab + lo, hi - lo,
                                          hipMemcpyHostToDevice, st) != hipSuccess)
                return 0;
            if (launch_groups(gs, g0, g1, (const unsigned char *)bp->d_tab, st, nullptr) != hipSuccess) return 0;
            return g1;
        };
        for (size_t a = 0, b = 0; a < groups.size() || b < groups2.size();) {
            if (a < groups.size() && (a = run_step(groups, a, stream)) == 0) {
                (void)hipGetLastError();
                return PA_DEVICE_ERROR;
            }
            if (b < groups2.size() && (b = run_step(groups2, b, bp->side)) == 0) {
                (void)hipGetLastError();
                return PA_DEVICE_ERROR;
            }
        }
        if (two && (hipEventRecord(bp->ev_join, bp->side) != hipSuccess ||
                    hipStreamWaitEvent(stream, bp->ev_join, 0) != hipSuccess)) {
            (void)hipGetLastError();
            return PA_DEVICE_ERROR;
        }
    } else {
        size_t lo, hi;
        fill_tables(groups, 0, groups.size(), bp->h_tab, &lo, &hi);
        // replay the captured list, or capture it now (its tables copied to a
        // buffer of its own first); `cap` runs after `stream`'s earlier work
        // and `stream` continues after the graph
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
            return PA_DEVICE_ERROR;
        if (!exec) {
            void *d_tab = nullptr;
            if (tab_bytes && (hipMalloc(&d_tab, tab_bytes) != hipSuccess ||
                              hipMemcpy(d_tab, bp->h_tab, tab_bytes, hipMemcpyHostToDevice) != hipSuccess)) {
                (void)hipGetLastError();
                if (d_tab) (void)hipFree(d_tab);
                return PA_ERR_NOMEM;
            }
            hipGraph_t graph = nullptr;
            if (hipStreamBeginCapture(bp->cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
                (void)hipFree(d_tab);
                return PA_DEVICE_ERROR;
            }
            const hipError_t el = launch_groups(groups, 0, groups.size(), (const unsigned char *)d_tab, bp->cap, bp);
            const hipError_t e = hipStreamEndCapture(bp->cap, &graph);
            hipError_t ei = hipErrorUnknown;
            if (el == hipSuccess && e == hipSuccess) ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                (void)hipGetLastError();
                (void)hipFree(d_tab);
                return PA_DEVICE_ERROR;
            }
            if (bp->graphs.size() >= kMaxGraphs) {
                // the evicted graph may still run: wait for the plan's work first
                if (hipStreamSynchronize(bp->cap) != hipSuccess) return PA_DEVICE_ERROR;
                (void)hipGraphExecDestroy(bp->graphs.front().exec);
                (void)hipFree(bp->graphs.front().d_tab);
                bp->graphs.erase(bp->graphs.begin());
            }
            bp->graphs.push_back(Captured{std::vector<pa_block>(blocks, blocks + count), bp->epoch, exec, d_tab});
        }
        if (hipGraphLaunch(exec, bp->cap) != hipSuccess || hipEventRecord(bp->ev_out, bp->cap) != hipSuccess ||
            hipStreamWaitEvent(stream, bp->ev_out, 0) != hipSuccess) {
            (void)hipGetLastError();
            return PA_DEVICE_ERROR;
        }
    }
    if (hipMemcpyAsync(bp->h_status, bp->d_status, (size_t)count * 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipGetLastError();
        return PA_DEVICE_ERROR;
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
