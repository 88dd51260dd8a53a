// Internal declarations shared by the libpa translation units.
//
// Arithmetic: exact number-theoretic transforms over the prime
// P = 2^64 - 2^32 + 1 ("Goldilocks"), whose multiplicative group has order
// 2^32 * 3 * 5 * 17 * 257 * 65537, so power-of-two lengths up to 2^32 exist.
// A gamma-bit number is cut into L = ceil(gamma/B) limbs of B bits (the
// paper's 2^B-ary words, Sec. 1 and Sec. 2.1); every coefficient of the sum of
// the k limb convolutions is below k*L*(2^B-1)^2, which the plan checks is
// below P, so the transform result is the exact integer coefficient.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "pa.h"

namespace pa {

constexpr uint64_t GL_P = 0xFFFFFFFF00000001ull;
constexpr uint64_t GL_EPS = 0xFFFFFFFFull;  // 2^64 mod P

// ---------------------------------------------------------------- field ops
// Values are kept canonical in [0, P).

__host__ __device__ __forceinline__ uint64_t gl_add(uint64_t a, uint64_t b) {
    uint64_t s = a + b;
    s = (s < a) ? s + GL_EPS : s;      // wrapped past 2^64: add 2^64 mod P
    s = (s >= GL_P) ? s - GL_P : s;
    return s;
}

__host__ __device__ __forceinline__ uint64_t gl_sub(uint64_t a, uint64_t b) {
    uint64_t d = a - b;
    d = (a < b) ? d - GL_EPS : d;      // borrowed 2^64: add P, i.e. subtract 2^64 - P
    return d;
}

// Reduce hi*2^64 + lo modulo P using 2^64 = 2^32 - 1 and 2^96 = -1 (mod P).
__host__ __device__ __forceinline__ uint64_t gl_reduce(uint64_t lo, uint64_t hi) {
    uint64_t hh = hi >> 32;
    uint64_t hl = hi & 0xFFFFFFFFull;
    uint64_t t0 = lo - hh;
    t0 = (lo < hh) ? t0 - GL_EPS : t0;
    uint64_t t1 = (hl << 32) - hl;
    uint64_t r = t0 + t1;
    r = (r < t1) ? r + GL_EPS : r;
    r = (r >= GL_P) ? r - GL_P : r;
    return r;
}

__host__ __device__ __forceinline__ uint64_t gl_mul(uint64_t a, uint64_t b) {
    uint64_t a0 = a & 0xFFFFFFFFull, a1 = a >> 32;
    uint64_t b0 = b & 0xFFFFFFFFull, b1 = b >> 32;
    uint64_t p00 = a0 * b0;
    uint64_t p01 = a0 * b1;
    uint64_t p10 = a1 * b0;
    uint64_t p11 = a1 * b1;
    uint64_t mid = (p00 >> 32) + (p01 & 0xFFFFFFFFull) + (p10 & 0xFFFFFFFFull);
    uint64_t lo = (mid << 32) | (p00 & 0xFFFFFFFFull);
    uint64_t hi = p11 + (p01 >> 32) + (p10 >> 32) + (mid >> 32);
    return gl_reduce(lo, hi);
}

__host__ __device__ __forceinline__ uint64_t gl_pow(uint64_t b, uint64_t e) {
    uint64_t r = 1;
    while (e) {
        if (e & 1) r = gl_mul(r, b);
        b = gl_mul(b, b);
        e >>= 1;
    }
    return r;
}

// ---------------------------------------------------------------- carry functions
// Carry transfer function of a run of limbs: carry_out = g + [carry_in >= th].
// th == CF_INF means the run's carry out does not depend on its carry in;
// g == CF_ID marks the identity (an empty run).
struct CFn {
    uint32_t g, th;
};
constexpr uint32_t CF_INF = 0xFFFFFFFFu;
constexpr uint32_t CF_ID = 0xFFFFFFFFu;

// Result block written by the tile-prefix kernel of a carry scan.
struct ScanResult {
    uint32_t carry_top[2];  // carry into the top limb for global carry-in 0 and 1
    uint32_t ov[2];         // value above the top limb's width for carry-in 0 and 1
    uint32_t sel;           // dual mode: 1 if the carry-in-1 variant is selected
    uint32_t final_carry;   // carry out of the last regular limb (carry-in 0)
    uint32_t pad[2];
};

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER_THREAD = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_PER_THREAD;

// Device status flag bits (written by the prologue and status kernels).
constexpr uint32_t ST_SEED_RANGE = 1u;
constexpr uint32_t ST_B_EVEN = 2u;
constexpr uint32_t ST_RELOAD = 4u;

}  // namespace pa

// ---------------------------------------------------------------- plan

struct pa_plan {
    int device;
    uint64_t n, r, gamma, k, L, N, W;
    uint64_t key_words, out_words;
    uint32_t B;
    uint32_t m, m1, m2, c_lg;   // N = 2^m = 2^m1 (column length) * 2^m2 (row length); 2^c_lg columns per tile
    uint32_t s_top;             // bits in the top limb: gamma - B*(L-1), in [1, B]
    uint32_t e_fold;            // B*L - gamma, in [0, B)
    uint64_t M1;                // digit count of the folded sum before reduction
    uint64_t ntiles_max;
    double exact_log2;

    // device memory (one allocation, carved)
    void *base;
    size_t workspace_bytes;
    uint64_t *X;        // 2k arrays of N words: column-pass outputs of x_i (0..k-1) and a_i (k..2k-1)
    uint64_t *Cc;       // N words: convolution coefficients
    uint32_t *t;        // digit sums (max(M1, L) + pad)
    uint32_t *s;        // normalised limbs of the folded sum (M1)
    uint32_t *y;        // MMH output limbs (L)
    uint32_t *U;        // MH value limbs (L)
    pa::CFn *agg;       // per-tile carry functions
    uint32_t *tcarry;   // per-tile carry-in, two variants
    pa::ScanResult *res;
    uint32_t *notones;  // k flags: chunk i has a limb that is not all ones
    uint32_t *status;   // seed/reload flags
    uint32_t *status_out;  // final flags of the last call (pa_hash reads it back)
    uint64_t *tw1f, *tw1i;  // omega_{N1}^j, omega_{N1}^-j, j < N1
    uint64_t *tw2f, *tw2i;  // omega_{N2}^j, omega_{N2}^-j, j < N2
    uint64_t *Wf, *Wi;      // four-step twiddles, row-major in stored (bit-reversed) row order
    uint32_t *h_status;     // pinned host word

    // phase profiling (pa_plan_set_profiling)
    int profiling;
    struct EvPair {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<EvPair> *pending;
    std::vector<hipEvent_t> *event_pool;
};

namespace pa {

// Kernel launchers (pa_kernels.hip).  All enqueue on `st` and return the
// first HIP error seen.
hipError_t launch_twiddles(pa_plan *p, hipStream_t st);
hipError_t launch_prologue(pa_plan *p, const uint64_t *a, const uint64_t *b, const uint64_t *c,
                           hipStream_t st);
hipError_t launch_mmh(pa_plan *p, const uint64_t *key, const uint64_t *a, hipStream_t st);
hipError_t launch_fold(pa_plan *p, hipStream_t st);
hipError_t launch_mh(pa_plan *p, const uint64_t *b, const uint64_t *c, hipStream_t st);
hipError_t launch_finish(pa_plan *p, uint64_t *out, uint32_t *d_status, uint64_t *y_out,
                         uint64_t *U_out, hipStream_t st);

// Marks the start or end of a phase on `st` when profiling is on (pa_api.cpp).
void phase_mark(pa_plan *p, int phase, bool begin, hipStream_t st);

}  // namespace pa
