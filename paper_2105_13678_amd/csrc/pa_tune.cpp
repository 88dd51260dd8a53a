// Autotuning of a block shape's plan: the limb width B (the paper's 2^B-ary
// words, Sec. 2.1), the transform length form (2^m or 3 * 2^m) and the
// column-tile width of the key-chunk column pass, chosen by timing every
// exact candidate on the device.  The output of a hash never depends on
// these choices, only its speed does.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "pa_internal.hpp"

namespace {

// splitmix64 (Steele, Lea, Flood, OOPSLA 2014): the random words of the
// timing inputs.
uint64_t mix64(uint64_t &state) {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Device buffers of one synthetic block: random key words and random seeds
// below 2^gamma with an odd b (valid inputs, so every candidate runs the
// whole sequence).
struct Inputs {
    uint64_t *key = nullptr, *a = nullptr, *b = nullptr, *c = nullptr, *out = nullptr;
    uint32_t *status = nullptr;
    bool ok = false;
    explicit Inputs(const pa_plan &p) {
        const size_t kw = p.key_words, aw = p.k * p.W, w = p.W, ow = p.out_words;
        ok = hipMalloc((void **)&key, kw * 8) == hipSuccess && hipMalloc((void **)&a, aw * 8) == hipSuccess &&
             hipMalloc((void **)&b, w * 8) == hipSuccess && hipMalloc((void **)&c, w * 8) == hipSuccess &&
             hipMalloc((void **)&out, ow * 8) == hipSuccess && hipMalloc((void **)&status, 4) == hipSuccess;
        if (!ok) return;
        uint64_t state = 0x5EEDull ^ p.n ^ (p.r << 20);
        const uint64_t top = (p.gamma & 63) ? (1ull << (p.gamma & 63)) - 1 : ~0ull;
        auto fill = [&](uint64_t *dst, size_t words, size_t chunk, bool odd) -> bool {
            std::vector<uint64_t> h(words);
            for (size_t i = 0; i < words; ++i) h[i] = mix64(state);
            if (chunk)
                for (size_t i = chunk - 1; i < words; i += chunk) h[i] &= top;
            if (odd && words) h[0] |= 1;
            return hipMemcpy(dst, h.data(), words * 8, hipMemcpyHostToDevice) == hipSuccess;
        };
        ok = fill(key, kw, 0, false) && fill(a, aw, w, false) && fill(b, w, w, true) && fill(c, w, w, false);
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

constexpr uint32_t kRounds = 5;  // rounds of the round-robin timing

}  // namespace

extern "C" {

pa_status pa_plan_tune(const pa_params *params, int hip_device, uint32_t reps, pa_params *best, double *best_ms) {
    if (!params || !best || reps == 0 || reps > 1000) return PA_ERR_ARG;
    pa_plan base{};
    pa::PlanLayout lay;
    pa_status st = pa::derive_plan(params, &base, &lay);
    if (st != PA_OK) return st;

    // candidates: for each admissible length form, the plan rule's limb width
    // for that form and the next narrower exact width that changes the
    // transform length (or the requested width), each with the rule's
    // column-tile width and its neighbours (or the requested tile width)
    std::vector<pa_params> cands;
    std::vector<pa_plan> shapes;
    const uint32_t forms[3] = {PA_FLAG_POW2_LENGTHS, PA_FLAG_RADIX3_LENGTHS, PA_FLAG_RADIX5_LENGTHS};
    for (uint32_t f : forms) {
        if (params->flags && params->flags != f) continue;
        pa_params q = *params;
        q.flags = f;
        q.col_lg = 0;
        pa_plan p0{};
        if (pa::derive_plan(&q, &p0, &lay) != PA_OK) continue;
        std::vector<uint32_t> widths{p0.B};
        if (!params->B)
            for (uint32_t b = p0.B - 1; b >= 8; --b) {
                q.B = b;
                pa_plan pb{};
                if (pa::derive_plan(&q, &pb, &lay) == PA_OK && pb.N != p0.N) {
                    widths.push_back(b);
                    break;
                }
            }
        for (uint32_t bw : widths) {
            q.B = bw;
            q.col_lg = 0;
            pa_plan pw{};
            if (pa::derive_plan(&q, &pw, &lay) != PA_OK) continue;
            const int c0 = (int)pw.c_lg;
            for (int dc = -1; dc <= 2; ++dc) {
                const int c = params->col_lg ? (int)params->col_lg : c0 + dc;
                if (params->col_lg && dc != 0) continue;
                if (c < 1) continue;
                q.col_lg = (uint32_t)c;
                pa_plan pc{};
                if (pa::derive_plan(&q, &pc, &lay) != PA_OK) continue;
                bool dup = false;
                for (const pa_plan &sh : shapes) dup |= same_shape(sh, pc);
                if (dup) continue;
                shapes.push_back(pc);
                cands.push_back(q);
            }
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
    // every candidate's plan first (one warm-up hash each), then kRounds
    // rounds that time each candidate in turn; a candidate's time is the
    // median of its rounds, so no candidate is favoured by its place in the
    // order
    std::vector<pa_plan *> plans(cands.size(), nullptr);
    pa_status result = PA_OK;
    bool any = false;
    for (size_t j = 0; j < cands.size() && result == PA_OK; ++j) {
        const pa_status cs = pa_plan_create(&cands[j], hip_device, &plans[j]);
        if (cs == PA_ERR_NOMEM) continue;  // too large for what is free now
        if (cs != PA_OK) {
            result = cs;
            break;
        }
        any = true;
        if (pa_hash_async(plans[j], in.key, in.a, in.b, in.c, in.out, in.status, s) != PA_OK) result = PA_ERR_DEVICE;
    }
    if (result == PA_OK && !any) result = PA_ERR_NOMEM;
    std::vector<std::vector<double>> times(cands.size());
    for (uint32_t round = 0; round < kRounds && result == PA_OK; ++round) {
        for (size_t j = 0; j < cands.size() && result == PA_OK; ++j) {
            if (!plans[j]) continue;
            bool ok = hipEventRecord(e0, s) == hipSuccess;
            for (uint32_t i = 0; ok && i < reps; ++i)
                ok = pa_hash_async(plans[j], in.key, in.a, in.b, in.c, in.out, in.status, s) == PA_OK;
            ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.f;
            ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            if (!ok) {
                (void)hipGetLastError();
                result = PA_ERR_DEVICE;
                break;
            }
            times[j].push_back((double)ms / reps);
        }
    }
    double best_t = 0.0;
    bool have = false;
    for (size_t j = 0; j < cands.size() && result == PA_OK; ++j) {
        if (times[j].empty()) continue;
        std::vector<double> &t = times[j];
        std::sort(t.begin(), t.end());
        const double med = t[t.size() / 2];
        if (!have || med < best_t) {
            have = true;
            best_t = med;
            *best = cands[j];
        }
    }
    for (pa_plan *pl : plans) pa_plan_destroy(pl);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    if (result == PA_OK && best_ms) *best_ms = best_t;
    return result;
}

}  // extern "C"
