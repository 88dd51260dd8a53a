// Device-side building blocks of the number-theoretic transforms over
// P = 2^64 - 2^32 + 1: field operations with the hardware carry chain,
// multiplication by constant powers of two, radix-2/4/8 butterflies and the
// LDS steps of a tile transform.
//
// Roots of unity: the plan picks omega_N so that omega_N^(N/64) = 8.  Then
// omega_8 = 2^24, omega_4 = 2^48 and omega_2 = 2^96 = -1, so every twiddle
// inside a radix-8 (or smaller) sub-transform is a power of two and costs a
// shift-and-reduce instead of a full 64x64-bit product.
#pragma once

#include "pa_internal.hpp"

namespace pa {

// ---------------------------------------------------------------- field ops
// All take and return canonical values in [0, P) unless stated otherwise.

__device__ __forceinline__ uint64_t fadd(uint64_t a, uint64_t b) {
    uint64_t s, t;
    bool c1 = __builtin_add_overflow(a, b, &s);
    bool c2 = __builtin_add_overflow(s, GL_EPS, &t);  // t = s - P (mod 2^64)
    return (c1 | c2) ? t : s;
}

__device__ __forceinline__ uint64_t fsub(uint64_t a, uint64_t b) {
    uint64_t d;
    bool c = __builtin_sub_overflow(a, b, &d);
    return c ? d - GL_EPS : d;  // wrapped: d + P (mod 2^64)
}

__device__ __forceinline__ uint64_t fneg(uint64_t a) { return a ? GL_P - a : 0ull; }

// hi*2^64 + lo mod P, for any hi, lo < 2^64; canonical result.
__device__ __forceinline__ uint64_t freduce(uint64_t lo, uint64_t hi) {
    const uint32_t r2 = (uint32_t)hi, r3 = (uint32_t)(hi >> 32);
    uint64_t t0;
    bool bo = __builtin_sub_overflow(lo, (uint64_t)r3, &t0);  // lo - hi_hi (2^96 = -1)
    t0 = bo ? t0 - GL_EPS : t0;
    const uint64_t u = ((uint64_t)r2 << 32) - r2;             // hi_lo * (2^32 - 1) (2^64 = 2^32 - 1)
    uint64_t r;
    bool c = __builtin_add_overflow(t0, u, &r);
    r = c ? r + GL_EPS : r;
    uint64_t q;
    bool c3 = __builtin_add_overflow(r, GL_EPS, &q);          // r >= P  <=>  r + 2^32 - 1 wraps
    return c3 ? q : r;
}

// Product of any two 64-bit values, reduced mod P (canonical).
__device__ __forceinline__ uint64_t fmul(uint64_t a, uint64_t b) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t p00 = (uint64_t)a0 * b0;
    const uint64_t t1 = (uint64_t)a0 * b1 + (p00 >> 32);
    const uint64_t t2 = (uint64_t)a1 * b0 + (uint32_t)t1;
    const uint64_t t3 = (uint64_t)a1 * b1 + (t1 >> 32);
    const uint64_t hi = t3 + (t2 >> 32);
    const uint64_t lo = (t2 << 32) | (uint32_t)p00;
    return freduce(lo, hi);
}

// x * 2^S mod P for a compile-time 0 < S < 96.
template <int S>
__device__ __forceinline__ uint64_t fmul_pow2(uint64_t x) {
    static_assert(S > 0 && S < 96, "shift out of range");
    if constexpr (S < 64) {
        return freduce(x << S, x >> (64 - S));
    } else {
        // x = xh*2^32 + xl; xh * 2^(S+32) = -xh * 2^(S-64) because 2^96 = -1
        const uint64_t xl = x & 0xFFFFFFFFull, xh = x >> 32;
        const uint64_t pos = freduce(0ull, xl << (S - 64));
        return fsub(pos, xh << (S - 64));  // xh * 2^(S-64) < 2^63 < P
    }
}

// ---------------------------------------------------------------- small DFTs
// Forward: natural order in, output slot s holds frequency bitrev(s).
// omega_8 = 2^24, omega_4 = 2^48.

__device__ __forceinline__ void bfly(uint64_t &u, uint64_t &v) {
    const uint64_t a = fadd(u, v), b = fsub(u, v);
    u = a;
    v = b;
}

template <int R>
__device__ __forceinline__ void dft_fwd(uint64_t *v);

template <>
__device__ __forceinline__ void dft_fwd<2>(uint64_t *v) {
    bfly(v[0], v[1]);
}

template <>
__device__ __forceinline__ void dft_fwd<4>(uint64_t *v) {
    bfly(v[0], v[2]);
    bfly(v[1], v[3]);
    v[3] = fmul_pow2<48>(v[3]);
    bfly(v[0], v[1]);
    bfly(v[2], v[3]);
}

template <>
__device__ __forceinline__ void dft_fwd<8>(uint64_t *v) {
    bfly(v[0], v[4]);
    bfly(v[1], v[5]);
    bfly(v[2], v[6]);
    bfly(v[3], v[7]);
    v[5] = fmul_pow2<24>(v[5]);
    v[6] = fmul_pow2<48>(v[6]);
    v[7] = fmul_pow2<72>(v[7]);
    bfly(v[0], v[2]);
    bfly(v[1], v[3]);
    bfly(v[4], v[6]);
    bfly(v[5], v[7]);
    v[3] = fmul_pow2<48>(v[3]);
    v[7] = fmul_pow2<48>(v[7]);
    bfly(v[0], v[1]);
    bfly(v[2], v[3]);
    bfly(v[4], v[5]);
    bfly(v[6], v[7]);
}

// Forward radix-8 DFT when v[4..7] are known to be zero (upper half of a
// zero-padded input): the first stage is v[j+4] = v[j] * omega_8^j.
__device__ __forceinline__ void dft_fwd8_lowhalf(uint64_t *v) {
    v[4] = v[0];
    v[5] = fmul_pow2<24>(v[1]);
    v[6] = fmul_pow2<48>(v[2]);
    v[7] = fmul_pow2<72>(v[3]);
    bfly(v[0], v[2]);
    bfly(v[1], v[3]);
    bfly(v[4], v[6]);
    bfly(v[5], v[7]);
    v[3] = fmul_pow2<48>(v[3]);
    v[7] = fmul_pow2<48>(v[7]);
    bfly(v[0], v[1]);
    bfly(v[2], v[3]);
    bfly(v[4], v[5]);
    bfly(v[6], v[7]);
}

// Inverse (without 1/R): input slot s holds frequency bitrev(s), natural
// order out.  omega^-1: omega_8^-1 = -2^72, omega_8^-2 = -2^48,
// omega_8^-3 = -2^24, omega_4^-1 = -2^48.  A negated twiddle swaps the
// butterfly's sum and difference.

// (u, v) -> (u - v, u + v): butterfly with twiddle -1 folded in
__device__ __forceinline__ void bfly_neg(uint64_t &u, uint64_t &v) {
    const uint64_t a = fsub(u, v), b = fadd(u, v);
    u = a;
    v = b;
}

template <int R>
__device__ __forceinline__ void dft_inv(uint64_t *v);

template <>
__device__ __forceinline__ void dft_inv<2>(uint64_t *v) {
    bfly(v[0], v[1]);
}

template <>
__device__ __forceinline__ void dft_inv<4>(uint64_t *v) {
    bfly(v[0], v[1]);
    bfly(v[2], v[3]);
    v[3] = fmul_pow2<48>(v[3]);
    bfly(v[0], v[2]);
    bfly_neg(v[1], v[3]);
}

template <>
__device__ __forceinline__ void dft_inv<8>(uint64_t *v) {
    bfly(v[0], v[1]);
    bfly(v[2], v[3]);
    bfly(v[4], v[5]);
    bfly(v[6], v[7]);
    v[3] = fmul_pow2<48>(v[3]);
    v[7] = fmul_pow2<48>(v[7]);
    bfly(v[0], v[2]);
    bfly_neg(v[1], v[3]);
    bfly(v[4], v[6]);
    bfly_neg(v[5], v[7]);
    v[5] = fmul_pow2<72>(v[5]);
    v[6] = fmul_pow2<48>(v[6]);
    v[7] = fmul_pow2<24>(v[7]);
    bfly(v[0], v[4]);
    bfly_neg(v[1], v[5]);
    bfly_neg(v[2], v[6]);
    bfly_neg(v[3], v[7]);
}

template <int R>
struct Lg;
template <>
struct Lg<2> {
    static constexpr int v = 1;
};
template <>
struct Lg<4> {
    static constexpr int v = 2;
};
template <>
struct Lg<8> {
    static constexpr int v = 3;
};

__device__ __forceinline__ uint32_t brev_small(uint32_t s, int bits) {
    return bits == 3 ? (((s & 1u) << 2) | (s & 2u) | ((s >> 2) & 1u)) : bits == 2 ? (((s & 1u) << 1) | ((s >> 1) & 1u)) : s;
}

// LDS swizzle: XOR the low 3 index bits with bits 5..7 so that the stride-8
// accesses of the last steps spread over all banks.  A bijection on any
// power-of-two range of at least 256 words and on every aligned 32-word block.
__device__ __forceinline__ uint32_t swz(uint32_t i) { return i ^ ((i >> 5) & 7u); }

// ---------------------------------------------------------------- tile steps
// A tile holds 2^cnt_lg interleaved transforms of length 2^lg: element
// (index, q) lives at buf[swz((index << cnt_lg) + q)].
//
// Forward step with radix R at sub-length M = 2^lgM (DIF, Cooley-Tukey): for
// each block b and n1 < M' = M/R the R values x[b*M + n1 + M'*n2] go through an
// R-point DFT; slot s (frequency k2 = bitrev(s)) is multiplied by
// omega_M^(n1*k2) and stored back at b*M + n1 + M'*s.  After all steps the
// transform sits in bit-reversed order.  tw[e] = omega_len^e, e < len.

template <int R, bool TW>
__device__ __forceinline__ void fwd_task(uint64_t *buf, uint32_t task, uint32_t lg, uint32_t lgM,
                                         uint32_t cnt_lg, const uint64_t *__restrict__ tw) {
    constexpr int LR = Lg<R>::v;
    const uint32_t lgMp = lgM - LR;
    const uint32_t q = task & ((1u << cnt_lg) - 1);
    const uint32_t rest = task >> cnt_lg;
    const uint32_t n1 = rest & ((1u << lgMp) - 1);
    const uint32_t base = ((rest >> lgMp) << lgM) + n1;
    uint64_t v[R];
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = buf[swz(((base + ((uint32_t)j << lgMp)) << cnt_lg) + q)];
    dft_fwd<R>(v);
    if (TW) {
#pragma unroll
        for (int s = 1; s < R; ++s)
            v[s] = fmul(v[s], tw[(n1 * brev_small(s, LR)) << (lg - lgM)]);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) buf[swz(((base + ((uint32_t)j << lgMp)) << cnt_lg) + q)] = v[j];
}

// Inverse of fwd_task: multiply slot s by omega_M^-(n1*k2), inverse R-point
// DFT, natural order back.  twi[e] = omega_len^-e.
template <int R, bool TW>
__device__ __forceinline__ void inv_task(uint64_t *buf, uint32_t task, uint32_t lg, uint32_t lgM,
                                         uint32_t cnt_lg, const uint64_t *__restrict__ twi) {
    constexpr int LR = Lg<R>::v;
    const uint32_t lgMp = lgM - LR;
    const uint32_t q = task & ((1u << cnt_lg) - 1);
    const uint32_t rest = task >> cnt_lg;
    const uint32_t n1 = rest & ((1u << lgMp) - 1);
    const uint32_t base = ((rest >> lgMp) << lgM) + n1;
    uint64_t v[R];
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = buf[swz(((base + ((uint32_t)j << lgMp)) << cnt_lg) + q)];
    if (TW) {
#pragma unroll
        for (int s = 1; s < R; ++s)
            v[s] = fmul(v[s], twi[(n1 * brev_small(s, LR)) << (lg - lgM)]);
    }
    dft_inv<R>(v);
#pragma unroll
    for (int j = 0; j < R; ++j) buf[swz(((base + ((uint32_t)j << lgMp)) << cnt_lg) + q)] = v[j];
}

template <int R, bool TW>
__device__ __forceinline__ void fwd_step(uint64_t *buf, uint32_t lg, uint32_t lgM, uint32_t cnt_lg,
                                         const uint64_t *__restrict__ tw, uint32_t tid, uint32_t nt) {
    const uint32_t ntask = (1u << (lg - Lg<R>::v)) << cnt_lg;
    for (uint32_t t = tid; t < ntask; t += nt) fwd_task<R, TW>(buf, t, lg, lgM, cnt_lg, tw);
    __syncthreads();
}

template <int R, bool TW>
__device__ __forceinline__ void inv_step(uint64_t *buf, uint32_t lg, uint32_t lgM, uint32_t cnt_lg,
                                         const uint64_t *__restrict__ twi, uint32_t tid, uint32_t nt) {
    const uint32_t ntask = (1u << (lg - Lg<R>::v)) << cnt_lg;
    for (uint32_t t = tid; t < ntask; t += nt) inv_task<R, TW>(buf, t, lg, lgM, cnt_lg, twi);
    __syncthreads();
}

// Steps of a length-2^lg transform: radix-8 at lgM = lg, lg-3, ... while at
// least 3 bits remain, then one radix-2 or radix-4 step at the bottom (whose
// twiddles are all 1).  Runs the steps from `first_lgM` down (forward).
__device__ __forceinline__ void fwd_steps_from(uint64_t *buf, uint32_t lg, uint32_t first_lgM, uint32_t cnt_lg,
                                               const uint64_t *__restrict__ tw, uint32_t tid, uint32_t nt) {
    uint32_t lgM = first_lgM;
    while (lgM >= 3) {
        if (lgM > 3)
            fwd_step<8, true>(buf, lg, lgM, cnt_lg, tw, tid, nt);
        else
            fwd_step<8, false>(buf, lg, lgM, cnt_lg, tw, tid, nt);
        lgM -= 3;
    }
    if (lgM == 2) fwd_step<4, false>(buf, lg, 2, cnt_lg, tw, tid, nt);
    if (lgM == 1) fwd_step<2, false>(buf, lg, 1, cnt_lg, tw, tid, nt);
}

// Inverse steps bottom-up, stopping after the step at `last_lgM`.
__device__ __forceinline__ void inv_steps_to(uint64_t *buf, uint32_t lg, uint32_t last_lgM, uint32_t cnt_lg,
                                             const uint64_t *__restrict__ twi, uint32_t tid, uint32_t nt) {
    const uint32_t r = lg % 3;
    if (r == 2) inv_step<4, false>(buf, lg, 2, cnt_lg, twi, tid, nt);
    if (r == 1) inv_step<2, false>(buf, lg, 1, cnt_lg, twi, tid, nt);
    for (uint32_t lgM = r + 3; lgM <= last_lgM; lgM += 3) {
        if (lgM > 3)
            inv_step<8, true>(buf, lg, lgM, cnt_lg, twi, tid, nt);
        else
            inv_step<8, false>(buf, lg, lgM, cnt_lg, twi, tid, nt);
    }
}

}  // namespace pa
