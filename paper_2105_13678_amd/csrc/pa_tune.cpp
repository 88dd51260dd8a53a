// Autotuning of a block shape's plan: the limb width B (the paper's 2^B-ary
// words, Sec. 2.1), the transform length form (2^m or 3 * 2^m) and the
// column-tile width of the key-chunk column pass, chosen by timing every
// exact candidate on the device.  The output of a hash never depends on
// these choices, only its speed does.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "pa_internal.hpp"

namespace {

// Device buffers of one synthetic block: all-zero key and seeds except an
// odd b (valid inputs; the kernels' work does not depend on the values).
struct Inputs {
    uint64_t *key = nullptr, *a = nullptr, *b = nullptr, *c = nullptr, *out = nullptr;
    uint32_t *status = nullptr;
    bool ok = false;
    Inputs(const pa_plan &p) {
        const size_t kw = p.key_words, aw = p.k * p.W, w = p.W, ow = p.out_words;
        ok = hipMalloc((void **)&key, kw * 8) == hipSuccess && hipMalloc((void **)&a, aw * 8) == hipSuccess &&
             hipMalloc((void **)&b, w * 8) == hipSuccess && hipMalloc((void **)&c, w * 8) == hipSuccess &&
             hipMalloc((void **)&out, ow * 8) == hipSuccess && hipMalloc((void **)&status, 4) == hipSuccess;
        const uint64_t one = 1;
        ok = ok && hipMemset(key, 0, kw * 8) == hipSuccess && hipMemset(a, 0, aw * 8) == hipSuccess &&
             hipMemset(b, 0, w * 8) == hipSuccess && hipMemset(c, 0, w * 8) == hipSuccess &&
             hipMemcpy(b, &one, 8, hipMemcpyHostToDevice) == hipSuccess;
    }
    ~Inputs() {
        for (void *q : {(void *)key, (void *)a, (void *)b, (void *)c, (void *)out, (void *)status})
            if (q) (void)hipFree(q);
        (void)hipGetLastError();
    }
};

bool same_shape(const pa_plan &x, const pa_plan &y) {
    return x.B == y.B && x.mix == y.mix && x.m == y.m && x.c_lg == y.c_lg;
}

}  // namespace

extern "C" {

pa_status pa_plan_tune(const pa_params *params, int hip_device, uint32_t reps, pa_params *best, double *best_ms) {
    if (!params || !best || reps == 0 || reps > 1000) return PA_ERR_ARG;
    pa_plan base{};
    pa::PlanLayout lay;
    pa_status st = pa::derive_plan(params, &base, &lay);
    if (st != PA_OK) return st;

    // candidates: for each admissible length form, the plan rule's limb width
    // (or the requested one) with the rule's column-tile width and its
    // neighbours (or the requested width)
    std::vector<pa_params> cands;
    std::vector<pa_plan> shapes;
    const uint32_t forms[2] = {PA_FLAG_POW2_LENGTHS, PA_FLAG_RADIX3_LENGTHS};
    for (uint32_t f : forms) {
        if (params->flags && params->flags != f) continue;
        pa_params q = *params;
        q.flags = f;
        q.col_lg = 0;
        pa_plan p0{};
        if (pa::derive_plan(&q, &p0, &lay) != PA_OK) continue;
        q.B = p0.B;
        const int c0 = (int)p0.c_lg;
        for (int dc = -1; dc <= 2; ++dc) {
            const int c = params->col_lg ? (int)params->col_lg : c0 + dc;
            if (params->col_lg && dc != 0) continue;
            if (c < 1) continue;
            q.col_lg = (uint32_t)c;
            pa_plan pc{};
            if (pa::derive_plan(&q, &pc, &lay) != PA_OK) continue;
            bool dup = false;
            for (const pa_plan &s : shapes) dup |= same_shape(s, pc);
            if (dup) continue;
            shapes.push_back(pc);
            cands.push_back(q);
        }
    }
    if (cands.empty()) return PA_ERR_INEXACT;

    pa::DeviceGuard guard(hip_device);
    if (!guard.ok) return PA_ERR_DEVICE;
    Inputs in(base);
    if (!in.ok) return PA_ERR_NOMEM;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (s) (void)hipStreamDestroy(s);
        if (e0) (void)hipEventDestroy(e0);
        (void)hipGetLastError();
        return PA_ERR_DEVICE;
    }
    pa_status result = PA_ERR_NOMEM;  // until one candidate has run
    double best_t = 0.0;
    for (const pa_params &q : cands) {
        pa_plan *plan = nullptr;
        const pa_status cs = pa_plan_create(&q, hip_device, &plan);
        if (cs == PA_ERR_NOMEM) continue;  // too large for what is free now
        if (cs != PA_OK) {
            result = cs;
            break;
        }
        bool ok = pa_hash_async(plan, in.key, in.a, in.b, in.c, in.out, in.status, s) == PA_OK;  // warm-up
        ok = ok && hipEventRecord(e0, s) == hipSuccess;
        for (uint32_t i = 0; ok && i < reps; ++i)
            ok = pa_hash_async(plan, in.key, in.a, in.b, in.c, in.out, in.status, s) == PA_OK;
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.f;
        ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        pa_plan_destroy(plan);
        if (!ok) {
            (void)hipGetLastError();
            result = PA_ERR_DEVICE;
            break;
        }
        const double t = (double)ms / reps;
        if (result != PA_OK || t < best_t) {
            result = PA_OK;
            best_t = t;
            *best = q;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    if (result == PA_OK && best_ms) *best_ms = best_t;
    return result;
}

}  // extern "C"
