// C interface of libpa: plan creation (parameter rule of Sec. 4 / Table 3 of
// arXiv 2105.13678), workspace layout and the per-block launch sequence.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "pa_internal.hpp"

namespace {

// Exponents e for which 2^e - 1 is a known Mersenne prime (the paper asks for
// p = M_gamma, Sec. 3.1 and Algorithm 1), increasing.
const uint64_t kMersenne[] = {
    2, 3, 5, 7, 13, 17, 19, 31, 61, 89, 107, 127, 521, 607, 1279, 2203, 2281,
    3217, 4253, 4423, 9689, 9941, 11213, 19937, 21701, 23209, 44497, 86243,
    110503, 132049, 216091, 756839, 859433, 1257787, 1398269, 2976221, 3021377,
    6972593, 13466917, 20996011, 24036583, 25964951, 30402457, 32582657,
    37156667, 42643801, 43112609, 57885161, 74207281, 77232917, 82589933,
    136279841};

constexpr uint64_t kMaxK = 4096;
// Lengths 3 * 2^m with m below this cost kMixSmallCost times their
// butterfly count in the plan rule (see derive_plan).
constexpr uint32_t kMinLog2Mix = 19;
constexpr double kMixSmallCost = 1.6;
// Lengths 5 * 2^m: their radix-5 passes (five inputs combined per column
// element, 16 products per coefficient in the reconstruction) count as
// kMix5Extra passes over N, and below 5 * 2^19 (generic column kernels only)
// kMix5SmallCost times the whole (device timings, candidates round robin:
// 5 * 2^19 and 5 * 2^20 take 0.92x and 0.89x the time of the 6/5 longer
// 3 * 2^20 and 3 * 2^21, 5 * 2^14 1.4x the time of the 8/5 longer 2^17).
constexpr double kMix5Extra = 3.0;
constexpr double kMix5SmallCost = 2.0;
constexpr double kLog2Of3 = 1.5849625007211562;
constexpr double kLog2Of5 = 2.321928094887362;
constexpr uint32_t kMinLog2N = 6;
constexpr uint32_t kMaxLdsLog2 = 14;  // 2^14 words = 64 KiB of LDS per tile

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

pa_status plan_shape(const pa_params *prm, uint64_t *gamma, uint64_t *k, uint32_t *B) {
    const uint32_t forms = PA_FLAG_POW2_LENGTHS | PA_FLAG_RADIX3_LENGTHS | PA_FLAG_RADIX5_LENGTHS;
    if (!prm || (prm->flags & ~forms) != 0 || (prm->flags & (prm->flags - 1)) != 0 || prm->reserved != 0)
        return PA_ERR_ARG;  // at most one length flag
    const uint64_t n = prm->n, r = prm->r;
    if (n < 2 || r < 1 || r >= n) return PA_ERR_ARG;
    uint64_t g = 0;
    if (prm->gamma == 0) {
        for (uint64_t e : kMersenne)
            if (e > r) {
                g = e;
                break;
            }
        if (!g) return PA_ERR_NO_GAMMA;
    } else {
        bool found = false;
        for (uint64_t e : kMersenne) found |= (e == prm->gamma);
        if (!found || prm->gamma <= r) return PA_ERR_GAMMA;
        g = prm->gamma;
    }
    if (prm->B != 0 && (prm->B < 8 || prm->B > 32)) return PA_ERR_ARG;
    *gamma = g;
    *k = (n + g - 1) / g;
    *B = prm->B;
    return PA_OK;
}

}  // namespace

extern "C" {

const char *pa_status_string(pa_status s) {
    switch (s) {
        case PA_OK: return "PA_OK";
        case PA_PENDING: return "PA_PENDING";
        case PA_RELOAD: return "PA_RELOAD";
        case PA_ERR_ARG: return "PA_ERR_ARG";
        case PA_ERR_NO_GAMMA: return "PA_ERR_NO_GAMMA";
        case PA_ERR_GAMMA: return "PA_ERR_GAMMA";
        case PA_ERR_INEXACT: return "PA_ERR_INEXACT";
        case PA_ERR_SEED_B_EVEN: return "PA_ERR_SEED_B_EVEN";
        case PA_ERR_SEED_RANGE: return "PA_ERR_SEED_RANGE";
        case PA_ERR_NOMEM: return "PA_ERR_NOMEM";
        case PA_ERR_DEVICE: return "PA_ERR_DEVICE";
        case PA_ERR_BUSY: return "PA_ERR_BUSY";
        case PA_ERR_LIMIT: return "PA_ERR_LIMIT";
    }
    return "PA_UNKNOWN";
}

pa_status pa_decode_status(uint32_t flags) {
    if (flags & pa::ST_SEED_RANGE) return PA_ERR_SEED_RANGE;
    if (flags & pa::ST_B_EVEN) return PA_ERR_SEED_B_EVEN;
    if (flags & pa::ST_RELOAD) return PA_RELOAD;
    return PA_OK;
}

}  // extern "C"

namespace {

// Transform length exponent for L limbs: the smallest m >= kMinLog2N with
// f * 2^m >= 2L - 1 (f = 1, 3 or 5; the full product of two L-limb numbers
// fits without wrap).
uint32_t log2_len(uint64_t L, uint32_t f = 1) {
    uint32_t m = kMinLog2N;
    while ((uint64_t)f << m < 2 * L - 1) ++m;
    return m;
}

// Prime triple for transforms of length 2^m (mix 0, m <= MAX_LOG2N), 3 * 2^m
// (mix 1, m <= MAX_LOG2N_MIX) or 5 * 2^m (mix 2, m <= MAX_LOG2N_MIX5); null
// beyond those lengths.
const pa::PrimeTriple *triple_for(uint32_t m, uint32_t mix) {
    if (mix == 2) {
        if (m > pa::MAX_LOG2N_MIX5) return nullptr;
        for (const pa::PrimeTriple &t : pa::PRIME_TRIPLES_5)
            if (m <= t.max_lg) return &t;
        return nullptr;
    }
    if (mix) {
        for (const pa::PrimeTriple &t : pa::PRIME_TRIPLES_3)
            if (m <= t.max_lg) return &t;
        return nullptr;
    }
    for (const pa::PrimeTriple &t : pa::PRIME_TRIPLES)
        if (m <= t.max_lg) return &t;
    return nullptr;
}

// Exactness of the three-prime transform: every coefficient of the sum of the
// k limb products is at most k*L*(2^B-1)^2 and must stay below p0*p1*p2.
bool exact(uint64_t k, uint64_t L, uint32_t B, const pa::PrimeTriple &T) {
    const unsigned __int128 P3 = (unsigned __int128)T.p[0] * T.p[1] * T.p[2];
    const unsigned __int128 lim = ((unsigned __int128)1 << B) - 1;
    const unsigned __int128 kL = (unsigned __int128)k * L;
    // kL < 2^37 (k <= kMaxK = 2^12, L < 2^25) and lim^2 < 2^64: the product fits in 128 bits
    return kL * lim * lim < P3;
}

}  // namespace

namespace pa {

// Derive every plan quantity from the request; no device access.
pa_status derive_plan(const pa_params *prm, pa_plan *p, PlanLayout *lay) {
    uint64_t gamma, k;
    uint32_t B;
    pa_status st = plan_shape(prm, &gamma, &k, &B);
    if (st != PA_OK) return st;
    if (k > kMaxK) return PA_ERR_LIMIT;
    // length forms tried: the flagged one, else all three
    const uint32_t mx_lo = (prm->flags & PA_FLAG_RADIX5_LENGTHS) ? 2u : (prm->flags & PA_FLAG_RADIX3_LENGTHS) ? 1u : 0u;
    const uint32_t mx_hi = (prm->flags & PA_FLAG_RADIX3_LENGTHS) ? 2u : (prm->flags & PA_FLAG_POW2_LENGTHS) ? 1u : 3u;
    // Candidate lengths for limb width b: the shortest 2^m, 3 * 2^m and
    // 5 * 2^m that hold the product, each with its own primes.  Cost model:
    // butterflies N log2 N, plus one pass over N for the radix-3 step
    // (kMix5Extra for the radix-5 step); lengths 3 * 2^m with m < kMinLog2Mix
    // count kMixSmallCost times that (timed on the device, candidates round
    // robin: at 3 * 2^10 ... 3 * 2^16 they take 1.06 - 1.24x the time of the
    // 4/3 longer power of two, at 3 * 2^19 the same, at 3 * 2^20 and 3 * 2^21
    // 0.92x and 0.56x), lengths 5 * 2^m kMix5SmallCost times.  `seen` records
    // whether some candidate length was within the supported range.
    bool seen = false;
    auto choose = [&](uint32_t b, uint32_t *m_out, uint32_t *mix_out, double *cost_out) {
        const uint64_t Lb = (gamma + b - 1) / b;
        bool ok = false;
        for (uint32_t mx = mx_lo; mx < mx_hi; ++mx) {
            const uint32_t f = pa::len_factor_of(mx);
            const uint32_t mb = log2_len(Lb, f);
            const pa::PrimeTriple *T = triple_for(mb, mx);
            if (!T) continue;
            seen = true;
            if (!exact(k, Lb, b, *T)) continue;
            const double Nl = (double)((uint64_t)f << mb);
            const double lgN = mb + (mx == 2 ? kLog2Of5 : mx ? kLog2Of3 : 0.0);
            const double extra = mx == 2 ? kMix5Extra : mx ? 1.0 : 0.0;
            const double small = mb >= kMinLog2Mix ? 1.0 : mx == 2 ? kMix5SmallCost : mx ? kMixSmallCost : 1.0;
            const double cost = Nl * (lgN + extra) * small;
            if (!ok || cost < *cost_out) {
                ok = true;
                *m_out = mb;
                *mix_out = mx;
                *cost_out = cost;
            }
        }
        return ok;
    };
    uint32_t m = 0, mix = 0;
    if (B == 0) {
        // cheapest exact transform over all limb widths, the widest among equals
        double best = 0.0;
        for (uint32_t b = 32; b >= 8; --b) {
            uint32_t mb, mx;
            double cost;
            if (choose(b, &mb, &mx, &cost) && (B == 0 || cost < best)) {
                B = b;
                m = mb;
                mix = mx;
                best = cost;
            }
        }
        if (B == 0) return seen ? PA_ERR_INEXACT : PA_ERR_LIMIT;
    } else {
        double cost;
        if (!choose(B, &m, &mix, &cost)) return seen ? PA_ERR_INEXACT : PA_ERR_LIMIT;
    }
    const uint64_t L = (gamma + B - 1) / B;
    const pa::PrimeTriple &T = *triple_for(m, mix);

    p->n = prm->n;
    p->r = prm->r;
    p->gamma = gamma;
    p->k = k;
    p->B = B;
    p->L = L;
    p->mix = mix;
    p->rf = pa::len_factor_of(mix);
    p->Nsub = 1ull << m;
    p->N = (uint64_t)p->rf << m;
    p->W = (gamma + 63) / 64;
    p->key_words = (prm->n + 63) / 64;
    p->out_words = (prm->r + 63) / 64;
    p->m = m;
    // rows of 2^m2 words (at most one 64 KiB LDS tile), columns of 2^m1 >= 8
    // words.  From N = 2^15 to 2^23 rows are 4096 words (three register
    // radix-16 steps); smaller transforms split about evenly; larger ones use
    // the longest LDS row.
    uint32_t m2;
    if (m >= 15 && m <= 23)
        m2 = 12;
    else if (m > 23)
        m2 = kMaxLdsLog2;
    else
        m2 = (m + 1) / 2;
    p->m2 = m2;
    p->m1 = m - m2;
    // Column tiles of 2^c columns x 2^m1 rows (at most 2^14 words of LDS).
    // The MH-stage forward pass (two arrays) uses 16 columns (64-byte row
    // segments; 8 for columns of 1024 rows), the single-array inverse pass 8
    // (more workgroups).  The
    // key-chunk pass widens short columns towards 256 first-step tasks per
    // tile (one per thread) while its 2k arrays still give at least 512
    // workgroups, and takes 8 columns of 1024 rows (4 first-step tasks per
    // thread; 16 such columns need the whole 64 KiB of LDS and about twice the
    // registers); a request may fix its width (col_lg, e.g. from pa_plan_tune).
    auto fit = [&](uint32_t c) {
        if (c > p->m2) c = p->m2;
        if (p->m1 + c > kMaxLdsLog2) c = kMaxLdsLog2 - p->m1;
        return c;
    };
    const uint32_t c_mh = fit(p->m1 == 10 ? 3 : 4);
    uint32_t c_mmh = fit(p->m1 < 7 ? 11 - p->m1 : p->m1 == 10 ? 3 : 4);
    while (c_mmh > c_mh && ((uint64_t)2 * k << (p->m2 - c_mmh)) < 512) --c_mmh;
    if (prm->col_lg) {
        if (prm->col_lg > p->m2 || p->m1 + prm->col_lg > kMaxLdsLog2) return PA_ERR_ARG;
        c_mmh = prm->col_lg;
    }
    p->c_lg = c_mmh;
    p->c_lg_mh = c_mh;
    p->ci_lg = c_mh < 3 ? c_mh : 3;
    p->s_top = (uint32_t)(gamma - (uint64_t)B * (L - 1));
    p->e_fold = (uint32_t)((uint64_t)B * L - gamma);
    const uint64_t Q = (96 + B - 1) / B, Q2 = (96 + p->e_fold + B - 1) / B;
    p->M1 = L + (Q > Q2 ? Q : Q2) + 1;
    const uint64_t digits = (p->M1 > L ? p->M1 : L) + 1;
    p->ntiles_max = (digits + pa::CARRY_TILE - 1) / pa::CARRY_TILE + 1;
    p->exact_log2 = std::log2((double)k) + std::log2((double)L) + 2.0 * std::log2((double)((1ull << B) - 1));
    pa::init_prime_constants(p, T.p);

    const size_t N = p->N, P3 = pa::NPRIMES;
    const size_t n1 = (size_t)1 << p->m1, n2 = (size_t)1 << p->m2;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    lay->oX = carve(2 * k * P3 * N * 4);
    lay->oC = carve(P3 * N * 4);
    lay->oC96 = carve(mix ? 3 * N * 4 : 0);
    lay->oT = carve(digits * 8);
    lay->oS = carve(p->M1 * 4);
    lay->oY = carve(L * 4);
    lay->oU = carve(L * 4);
    lay->oAgg = carve(2 * p->ntiles_max * sizeof(pa::CFn));  // fold and wrap chains
    lay->oNo = carve((k << p->m2) * 4);  // reload flags per key chunk and column tile (at most 2^m2)
    lay->oTf = carve(p->ntiles_max * 4);
    lay->oSt = carve(4 * 4);
    lay->oSo = carve(4 * 4);
    lay->scratch_bytes = off;
    lay->oT1 = carve(P3 * n1 * 4 * 2);
    lay->oT2 = carve(P3 * n2 * 4 * 2);
    lay->oW = carve(P3 * N * 4 * 2);
    lay->oR16 = carve(P3 * pa::R16_TW * 4 * 2);
    // radix-3 / radix-5 row twiddles: (f + 1) / 2 forward tables and one inverse table,
    // each NPRIMES x f x N1 words
    lay->oG3 = carve(mix ? (size_t)((p->rf + 1) / 2 + 1) * P3 * p->rf * n1 * 4 : 0);
    lay->total = off;
    lay->table_bytes = off - lay->scratch_bytes;
    p->workspace_bytes = off;
    p->scratch_bytes = lay->scratch_bytes;
    return PA_OK;
}

void bind_scratch(pa_plan *p, void *scratch, const PlanLayout &lay) {
    char *b = (char *)scratch;
    p->X = (uint32_t *)(b + lay.oX);
    p->Cc = (uint32_t *)(b + lay.oC);
    p->C96 = (uint32_t *)(b + lay.oC96);
    p->t = (uint64_t *)(b + lay.oT);
    p->s = (uint32_t *)(b + lay.oS);
    p->y = (uint32_t *)(b + lay.oY);
    p->U = (uint32_t *)(b + lay.oU);
    p->agg = (pa::CFn *)(b + lay.oAgg);
    p->agg_w = p->agg + p->ntiles_max;
    p->notones = (uint32_t *)(b + lay.oNo);
    p->status = (uint32_t *)(b + lay.oSt);
    p->tflags = (uint32_t *)(b + lay.oTf);
    p->status_out = (uint32_t *)(b + lay.oSo);
}

void bind_tables(pa_plan *p, void *tables, const PlanLayout &lay) {
    char *b = (char *)tables - lay.scratch_bytes;  // table offsets follow the scratch
    const size_t N = p->N, P3 = pa::NPRIMES;
    const size_t n1 = (size_t)1 << p->m1, n2 = (size_t)1 << p->m2;
    p->tw1f = (uint32_t *)(b + lay.oT1);
    p->tw1i = p->tw1f + P3 * n1;
    p->tw2f = (uint32_t *)(b + lay.oT2);
    p->tw2i = p->tw2f + P3 * n2;
    p->Wf = (uint32_t *)(b + lay.oW);
    p->Wi = p->Wf + P3 * N;
    p->R16f = (uint32_t *)(b + lay.oR16);
    p->R16i = p->R16f + P3 * pa::R16_TW;
    p->G3 = p->mix ? (uint32_t *)(b + lay.oG3) : nullptr;
}

pa_status enqueue_hash(pa_plan *p, const uint64_t *key, const uint64_t *a, const uint64_t *b,
                       const uint64_t *c, uint64_t *out, uint32_t *d_status, uint64_t *y_out,
                       uint64_t *U_out, hipStream_t st) {
    if (!p || !key || !a || !b || !c || !out) return PA_ERR_ARG;
    hipError_t e = pa::launch_mmh(p, key, a, st);
    if (e == hipSuccess) e = pa::launch_fold(p, pa::Seeds{a, b, c}, st);
    if (e == hipSuccess) e = pa::launch_mh(p, b, c, out, d_status, st);
    // y as an output: the second fold's general case, if flagged, after the MH stage
    if (e == hipSuccess && y_out && pa::wrap_inline(p)) e = pa::launch_wrap(p, st);
    if (e == hipSuccess && (y_out || U_out)) e = pa::launch_finish(p, y_out, U_out, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return PA_ERR_DEVICE;
    }
    return PA_OK;
}

}  // namespace pa

extern "C" {

pa_status pa_plan_query(const pa_params *prm, pa_plan_info *info) {
    if (!info) return PA_ERR_ARG;
    pa_plan tmp{};
    pa::PlanLayout lay;
    pa_status st = pa::derive_plan(prm, &tmp, &lay);
    if (st != PA_OK) return st;
    return pa_plan_get_info(&tmp, info);
}

pa_status pa_plan_create(const pa_params *prm, int hip_device, pa_plan **out) {
    if (!out) return PA_ERR_ARG;
    *out = nullptr;
    pa_plan *p = new (std::nothrow) pa_plan();
    if (!p) return PA_ERR_NOMEM;
    pa::PlanLayout lay;
    pa_status st = pa::derive_plan(prm, p, &lay);
    if (st != PA_OK) {
        delete p;
        return st;
    }
    p->device = hip_device;

    pa::DeviceGuard guard(hip_device);
    if (!guard.ok) {
        delete p;
        return PA_ERR_DEVICE;
    }
    if (hipMalloc(&p->base, lay.total) != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return PA_ERR_NOMEM;
    }
    if (hipHostMalloc((void **)&p->h_status, 64, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(p->base);
        delete p;
        return PA_ERR_NOMEM;
    }
    pa::bind_scratch(p, p->base, lay);
    pa::bind_tables(p, (char *)p->base + lay.scratch_bytes, lay);

    hipStream_t s0 = nullptr;
    if (pa::launch_twiddles(p, s0) != hipSuccess || hipStreamSynchronize(s0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(p->h_status);
        (void)hipFree(p->base);
        delete p;
        return PA_ERR_DEVICE;
    }
    *out = p;
    return PA_OK;
}

pa_status pa_plan_fill_scratch(pa_plan *p, uint32_t word, hipStream_t stream) {
    if (!p) return PA_ERR_ARG;
    pa::DeviceGuard guard(p->device);
    if (!guard.ok) return PA_ERR_DEVICE;
    if (pa::launch_fill((uint32_t *)p->base, p->scratch_bytes / 4, word, stream) != hipSuccess) {
        (void)hipGetLastError();
        return PA_ERR_DEVICE;
    }
    return PA_OK;
}

pa_status pa_plan_get_info(const pa_plan *p, pa_plan_info *info) {
    if (!p || !info) return PA_ERR_ARG;
    std::memset(info, 0, sizeof(*info));
    info->n = p->n;
    info->r = p->r;
    info->gamma = p->gamma;
    info->k = p->k;
    info->B = p->B;
    info->log2N = p->m;
    info->L = p->L;
    info->N = p->N;
    info->key_words = p->key_words;
    info->seed_words = p->W;
    info->a_words = p->k * p->W;
    info->out_words = p->out_words;
    info->workspace_bytes = p->workspace_bytes;
    info->exact_log2 = p->exact_log2;
    info->log2N1 = p->m1;
    info->log2N2 = p->m2;
    info->nprimes = pa::NPRIMES;
    for (int q = 0; q < pa::NPRIMES; ++q) info->primes[q] = p->primes.c[q].p;
    info->len_factor = p->rf;
    info->col_lg = p->c_lg;
    return PA_OK;
}

void pa_plan_destroy(pa_plan *p) {
    if (!p) return;
    pa::DeviceGuard guard(p->device);
    (void)hipDeviceSynchronize();
    if (p->pending) {
        for (auto &e : *p->pending) {
            (void)hipEventDestroy(e.a);
            if (e.b) (void)hipEventDestroy(e.b);
        }
        delete p->pending;
    }
    if (p->event_pool) {
        for (auto e : *p->event_pool) (void)hipEventDestroy(e);
        delete p->event_pool;
    }
    (void)hipHostFree(p->h_status);
    (void)hipFree(p->base);
    delete p;
}

pa_status pa_plan_set_profiling(pa_plan *p, uint32_t phase_mask) {
    if (!p) return PA_ERR_ARG;
    if (!p->pending) p->pending = new (std::nothrow) std::vector<pa_plan::EvPair>();
    if (!p->event_pool) p->event_pool = new (std::nothrow) std::vector<hipEvent_t>();
    if (!p->pending || !p->event_pool) return PA_ERR_NOMEM;
    if (phase_mask & ~PA_PROFILE_ALL) return PA_ERR_ARG;
    p->profiling = phase_mask;
    return PA_OK;
}

pa_status pa_plan_read_profile(pa_plan *p, double *ms, uint64_t *calls) {
    if (!p || !ms || !calls) return PA_ERR_ARG;
    for (int i = 0; i < PA_PH_COUNT; ++i) {
        ms[i] = 0.0;
        calls[i] = 0;
    }
    if (!p->pending) return PA_OK;
    pa::DeviceGuard guard(p->device);
    pa_status st = PA_OK;
    for (auto &e : *p->pending) {
        float t = 0.f;
        if (!e.b || hipEventSynchronize(e.b) != hipSuccess || hipEventElapsedTime(&t, e.a, e.b) != hipSuccess) {
            (void)hipGetLastError();
            st = PA_ERR_DEVICE;
        } else {
            ms[e.phase] += t;
            calls[e.phase] += 1;
        }
        p->event_pool->push_back(e.a);
        if (e.b) p->event_pool->push_back(e.b);
    }
    p->pending->clear();
    return st;
}

static pa_status wait_status(pa_plan *p, hipStream_t st) {
    if (hipMemcpyAsync(p->h_status, p->status_out, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        return PA_ERR_DEVICE;
    }
    return pa_decode_status(*p->h_status);
}

pa_status pa_hash(pa_plan *p, const uint64_t *key, const uint64_t *a, const uint64_t *b, const uint64_t *c,
                  uint64_t *out, hipStream_t st) {
    if (!p) return PA_ERR_ARG;
    pa::DeviceGuard guard(p->device);
    if (!guard.ok) return PA_ERR_DEVICE;
    pa_status s = pa::enqueue_hash(p, key, a, b, c, out, nullptr, nullptr, nullptr, st);
    if (s != PA_OK) return s;
    return wait_status(p, st);
}

pa_status pa_hash_async(pa_plan *p, const uint64_t *key, const uint64_t *a, const uint64_t *b,
                        const uint64_t *c, uint64_t *out, uint32_t *d_status, hipStream_t st) {
    if (!p || !d_status) return PA_ERR_ARG;
    pa::DeviceGuard guard(p->device);
    if (!guard.ok) return PA_ERR_DEVICE;
    return pa::enqueue_hash(p, key, a, b, c, out, d_status, nullptr, nullptr, st);
}

pa_status pa_hash_stages(pa_plan *p, const uint64_t *key, const uint64_t *a, const uint64_t *b,
                         const uint64_t *c, uint64_t *out, uint64_t *y_out, uint64_t *U_out,
                         hipStream_t st) {
    if (!p || !y_out || !U_out) return PA_ERR_ARG;
    pa::DeviceGuard guard(p->device);
    if (!guard.ok) return PA_ERR_DEVICE;
    pa_status s = pa::enqueue_hash(p, key, a, b, c, out, nullptr, y_out, U_out, st);
    if (s != PA_OK) return s;
    return wait_status(p, st);
}

}  // extern "C"

namespace pa {

void phase_mark(pa_plan *p, int phase, bool begin, hipStream_t st) {
    if (!(p->profiling >> phase & 1u) || !p->pending || !p->event_pool) return;
    hipEvent_t ev;
    if (!p->event_pool->empty()) {
        ev = p->event_pool->back();
        p->event_pool->pop_back();
    } else if (hipEventCreate(&ev) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    if (hipEventRecord(ev, st) != hipSuccess) {
        (void)hipGetLastError();
        p->event_pool->push_back(ev);
        return;
    }
    if (begin) {
        p->pending->push_back(pa_plan::EvPair{phase, ev, nullptr});
    } else if (!p->pending->empty() && p->pending->back().phase == phase && !p->pending->back().b) {
        p->pending->back().b = ev;
    } else {
        p->event_pool->push_back(ev);
    }
}

}  // namespace pa
