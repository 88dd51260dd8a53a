// Device building blocks of the number-theoretic transforms: Montgomery
// arithmetic modulo three primes below 2^30, radix-2/4/8/16 butterflies and
// the LDS steps of a tile transform.
//
// Lazy residues.  Because every prime satisfies 4p < 2^32, transform values
// are kept only partially reduced: forward-transform values lie in [0, 2p),
// inverse-transform values in [0, 4p).  The Montgomery product (R = 2^32) of
// a and b with a*b < 2^32 p is (a*b + m*p) / 2^32 < 2p with m = (a*b)(-1/p)
// mod 2^32: three full-rate VALU instructions on gfx950 (v_mad_u64_u32,
// v_mul_lo_u32, v_mad_u64_u32), no final subtraction.  A radix-2 butterfly
// is then eight instructions (sum and its reduction to [0, 2p): 3; the
// difference shifted by 2p: 2; the product: 3).  Canonical values [0, p) are
// produced only where a consumer needs them (the Chinese-remainder step).
#pragma once

#include "pa_internal.hpp"

namespace pa {

// ---------------------------------------------------------------- field ops

// a * b * 2^-32 mod p, in [0, 2p); requires a * b < 2^32 p (e.g. a < 4p and
// b < p, or a, b < 2p).
__device__ __forceinline__ uint32_t mont(uint32_t a, uint32_t b, const PrimeConst &M) {
    const uint64_t t = (uint64_t)a * b;
    const uint32_t m = (uint32_t)t * M.pinv;
    return (uint32_t)(((uint64_t)m * M.p + t) >> 32);  // t + m p < 2^33 p < 2^64, divisible by 2^32
}

// T * 2^-32 mod p for a 64-bit T < 2^64 - 2^32 p (Montgomery reduction of a
// sum of raw products); the result is below T / 2^32 + p.
__device__ __forceinline__ uint32_t redc64(uint64_t T, const PrimeConst &M) {
    const uint32_t m = (uint32_t)T * M.pinv;
    return (uint32_t)((T + (uint64_t)m * M.p) >> 32);
}

// [0, 4p) -> [0, 2p), same residue
__device__ __forceinline__ uint32_t red2(uint32_t x, const PrimeConst &M) { return min(x, x - M.p2); }

// [0, 2p) -> [0, p), same residue
__device__ __forceinline__ uint32_t canon(uint32_t x, const PrimeConst &M) { return min(x, x - M.p); }

// canonical a * b * 2^-32 mod p, for a < 2^32 and b < p
__device__ __forceinline__ uint32_t mmul(uint32_t a, uint32_t b, const PrimeConst &M) {
    return canon(mont(a, b, M), M);
}

// canonical sum and difference of canonical values
__device__ __forceinline__ uint32_t madd(uint32_t a, uint32_t b, const PrimeConst &M) {
    const uint32_t s = a + b;
    return min(s, s - M.p);
}

__device__ __forceinline__ uint32_t msub(uint32_t a, uint32_t b, const PrimeConst &M) {
    const uint32_t d = a - b;
    return min(d, d + M.p);
}

// ---------------------------------------------------------------- small DFTs
// R-point DFTs (R = 2, 4, 8, 16) as log2(R) radix-2 stages in registers.
//
// Forward (decimation in frequency), values in [0, 2p): natural order in,
// output slot s holds frequency bitrev(s).  The stage with half-size h
// multiplies the difference at offset j by omega_{2h}^j = M.w16[j*8/h].
// With TW, output slot s (s >= 1) is also multiplied by tw[s] (a step
// twiddle, canonical Montgomery form); the multiplication is fused into the
// last stage, whose unreduced sum and difference (< 4p) go straight into the
// product.  With LOWHALF the upper half of the input is known to be zero, so
// the first stage is v[j + R/2] = v[j] * omega_R^j.
template <int R, bool LOWHALF, bool TW>
__device__ __forceinline__ void dft_fwd_x(uint32_t *v, const uint32_t *tw, const PrimeConst &M) {
    static_assert(!LOWHALF || R >= 4, "the zero-upper-half form needs a second stage");
    constexpr int H = R / 2;
    if (LOWHALF) {
#pragma unroll
        for (int j = 0; j < H; ++j) v[j + H] = j ? mont(v[j], M.w16[j * (8 / H)], M) : v[j];
    }
#pragma unroll
    for (int h = LOWHALF ? H / 2 : H; h >= 1; h >>= 1) {
#pragma unroll
        for (int blk = 0; blk < R; blk += 2 * h) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                const uint32_t u = v[blk + j], x = v[blk + j + h];
                const uint32_t sum = u + x;           // < 4p
                const uint32_t dif = u + M.p2 - x;    // (0, 4p)
                if (TW && h == 1) {
                    v[blk] = blk ? mont(sum, tw[blk], M) : red2(sum, M);
                    v[blk + 1] = mont(dif, tw[blk + 1], M);
                } else {
                    v[blk + j] = red2(sum, M);
                    v[blk + j + h] = j ? mont(dif, M.w16[j * (8 / h)], M) : red2(dif, M);
                }
            }
        }
    }
}

template <int R>
__device__ __forceinline__ void dft_fwd(uint32_t *v, const PrimeConst &M) {
    dft_fwd_x<R, false, false>(v, nullptr, M);
}

template <int R>
__device__ __forceinline__ void dft_fwd_tw(uint32_t *v, const uint32_t *tw, const PrimeConst &M) {
    dft_fwd_x<R, false, true>(v, tw, M);
}

// Inverse (times R), values in [0, 4p): undoes the forward stages in reverse
// order with omega^-1 (M.w16i); bit-reversed slots in, natural order out.
// With TW, input slot s (s >= 1) is first multiplied by tw[s], fused into the
// first stage.
template <int R, bool TW>
__device__ __forceinline__ void dft_inv_x(uint32_t *v, const uint32_t *tw, const PrimeConst &M) {
#pragma unroll
    for (int h = 1; h < R; h <<= 1) {
#pragma unroll
        for (int blk = 0; blk < R; blk += 2 * h) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                uint32_t a, q;  // both < 2p
                if (TW && h == 1) {
                    a = blk ? mont(v[blk], tw[blk], M) : red2(v[blk], M);
                    q = mont(v[blk + 1], tw[blk + 1], M);
                } else {
                    a = red2(v[blk + j], M);
                    q = j ? mont(v[blk + j + h], M.w16i[j * (8 / h)], M) : red2(v[blk + j + h], M);
                }
                v[blk + j] = a + q;             // < 4p
                v[blk + j + h] = a + M.p2 - q;  // (0, 4p)
            }
        }
    }
}

template <int R>
__device__ __forceinline__ void dft_inv(uint32_t *v, const PrimeConst &M) {
    dft_inv_x<R, false>(v, nullptr, M);
}

template <int R>
__device__ __forceinline__ void dft_inv_tw(uint32_t *v, const uint32_t *tw, const PrimeConst &M) {
    dft_inv_x<R, true>(v, tw, M);
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
template <>
struct Lg<16> {
    static constexpr int v = 4;
};

// bit reversal of s within `bits` bits (bits <= 4; constant-folded in unrolled loops)
__device__ __forceinline__ constexpr uint32_t brev_small(uint32_t s, int bits) {
    uint32_t r = 0;
    for (int i = 0; i < bits; ++i) r |= ((s >> i) & 1u) << (bits - 1 - i);
    return r;
}

// LDS swizzle for 32-bit elements: bits 6..8 of the index are XORed into
// bits 0..2 and 3..5.  An involution that permutes each aligned 64-element
// block, chosen so that the stride-8 accesses of the last radix-8 step and
// the stride-64/8 pattern of the step before it hit 64 distinct banks.
__device__ __forceinline__ uint32_t swz(uint32_t i) {
    const uint32_t v = (i >> 6) & 7u;
    return i ^ (v | (v << 3));
}

// Swizzle of a tile of 2^cnt_lg interleaved transforms (cnt_lg > 0): bits
// [cnt_lg + 3, cnt_lg + 3 + w) are XORed into bits [cnt_lg, cnt_lg + w),
// w = 6 - cnt_lg, so that the last radix-8 step (a wave covers all columns
// of 64 / 2^cnt_lg consecutive 8-row blocks) touches 64 distinct banks.
// Triangular in the bit order, hence a bijection on any 2^n-word tile.
__device__ __forceinline__ uint32_t tile_swz(uint32_t i, uint32_t cnt_lg) {
    if (cnt_lg == 0) return swz(i);
    if (cnt_lg >= 6) return i;
    const uint32_t w = 6 - cnt_lg;
    return i ^ (((i >> (cnt_lg + 3)) & ((1u << w) - 1)) << cnt_lg);
}

// ---------------------------------------------------------------- tile steps
// A tile holds 2^cnt_lg interleaved transforms of length 2^lg: element
// (index, q) lives at buf[tile_swz((index << cnt_lg) + q, cnt_lg)].
//
// Forward step with radix R at sub-length M = 2^lgM (decimation in
// frequency, values in [0, 2p)): for each block b and n1 < M' = M/R, the R values
// x[b*M + n1 + M'*n2] go through an R-point DFT; slot s (frequency
// k2 = bitrev(s)) is multiplied by omega_M^(n1*k2) and stored back at
// b*M + n1 + M'*s.  After all steps the transform is in bit-reversed order.
// tw[e] = omega_len^e (Montgomery form), e < len.

template <int R, bool TW>
__device__ __forceinline__ void fwd_task(uint32_t *buf, uint32_t task, uint32_t lg, uint32_t lgM,
                                         uint32_t cnt_lg, const uint32_t *__restrict__ tw, const PrimeConst &M) {
    constexpr int LR = Lg<R>::v;
    const uint32_t lgMp = lgM - LR;
    const uint32_t q = task & ((1u << cnt_lg) - 1);
    const uint32_t rest = task >> cnt_lg;
    const uint32_t n1 = rest & ((1u << lgMp) - 1);
    const uint32_t base = ((rest >> lgMp) << lgM) + n1;
    uint32_t v[R], w[R];
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = buf[tile_swz(((base + ((uint32_t)j << lgMp)) << cnt_lg) + q, cnt_lg)];
    if (TW) {
#pragma unroll
        for (int s = 1; s < R; ++s) w[s] = tw[(n1 * brev_small(s, LR)) << (lg - lgM)];
    }
    dft_fwd_x<R, false, TW>(v, w, M);
#pragma unroll
    for (int j = 0; j < R; ++j) buf[tile_swz(((base + ((uint32_t)j << lgMp)) << cnt_lg) + q, cnt_lg)] = v[j];
}

// Inverse of fwd_task (values in [0, 4p)): multiply slot s by
// omega_M^-(n1*k2), inverse R-point DFT, natural order back.
// twi[e] = omega_len^-e.
template <int R, bool TW>
__device__ __forceinline__ void inv_task(uint32_t *buf, uint32_t task, uint32_t lg, uint32_t lgM,
                                         uint32_t cnt_lg, const uint32_t *__restrict__ twi, const PrimeConst &M) {
    constexpr int LR = Lg<R>::v;
    const uint32_t lgMp = lgM - LR;
    const uint32_t q = task & ((1u << cnt_lg) - 1);
    const uint32_t rest = task >> cnt_lg;
    const uint32_t n1 = rest & ((1u << lgMp) - 1);
    const uint32_t base = ((rest >> lgMp) << lgM) + n1;
    uint32_t v[R], w[R];
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = buf[tile_swz(((base + ((uint32_t)j << lgMp)) << cnt_lg) + q, cnt_lg)];
    if (TW) {
#pragma unroll
        for (int s = 1; s < R; ++s) w[s] = twi[(n1 * brev_small(s, LR)) << (lg - lgM)];
    }
    dft_inv_x<R, TW>(v, w, M);
#pragma unroll
    for (int j = 0; j < R; ++j) buf[tile_swz(((base + ((uint32_t)j << lgMp)) << cnt_lg) + q, cnt_lg)] = v[j];
}

// The synchronisation between two LDS steps: the workgroup's barrier, or
// (WS) only the calling wavefront's, when every thread that shares the
// buffer is in that wavefront: its LDS accesses are then ordered by the
// wavefront-scope fences alone.
template <bool WS>
__device__ __forceinline__ void step_sync() {
    if constexpr (WS) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <int R, bool TW, bool WS = false>
__device__ __forceinline__ void fwd_step(uint32_t *buf, uint32_t lg, uint32_t lgM, uint32_t cnt_lg,
                                         const uint32_t *__restrict__ tw, const PrimeConst &M, uint32_t tid,
                                         uint32_t nt) {
    const uint32_t ntask = (1u << (lg - Lg<R>::v)) << cnt_lg;
    for (uint32_t t = tid; t < ntask; t += nt) fwd_task<R, TW>(buf, t, lg, lgM, cnt_lg, tw, M);
    step_sync<WS>();
}

template <int R, bool TW, bool WS = false>
__device__ __forceinline__ void inv_step(uint32_t *buf, uint32_t lg, uint32_t lgM, uint32_t cnt_lg,
                                         const uint32_t *__restrict__ twi, const PrimeConst &M, uint32_t tid,
                                         uint32_t nt) {
    const uint32_t ntask = (1u << (lg - Lg<R>::v)) << cnt_lg;
    for (uint32_t t = tid; t < ntask; t += nt) inv_task<R, TW>(buf, t, lg, lgM, cnt_lg, twi, M);
    step_sync<WS>();
}

// Sub-length of the last (twiddle-free) step of a length-2^lg transform:
// radix 8 at 2^3 when 3 divides lg, else radix 2 at 2^1 or radix 4 at 2^2.
__device__ __forceinline__ uint32_t last_lgM(uint32_t lg) {
    const uint32_t r = lg % 3;
    return r == 0 ? 3u : r;
}

// Forward radix-8 steps with twiddles from sub-length 2^from_lgM down to
// 2^(last_lgM(lg) + 3), i.e. everything between a first and a last step.
__device__ __forceinline__ void fwd_middle_steps(uint32_t *buf, uint32_t lg, uint32_t from_lgM, uint32_t cnt_lg,
                                                 const uint32_t *__restrict__ tw, const PrimeConst &M,
                                                 uint32_t tid, uint32_t nt) {
    for (uint32_t lgM = from_lgM; lgM > last_lgM(lg); lgM -= 3) fwd_step<8, true>(buf, lg, lgM, cnt_lg, tw, M, tid, nt);
}

// Inverse radix-8 steps with twiddles from sub-length 2^(last_lgM(lg) + 3) up
// to 2^to_lgM.
__device__ __forceinline__ void inv_middle_steps(uint32_t *buf, uint32_t lg, uint32_t to_lgM, uint32_t cnt_lg,
                                                 const uint32_t *__restrict__ twi, const PrimeConst &M,
                                                 uint32_t tid, uint32_t nt) {
    for (uint32_t lgM = last_lgM(lg) + 3; lgM <= to_lgM; lgM += 3) inv_step<8, true>(buf, lg, lgM, cnt_lg, twi, M, tid, nt);
}

// Forward steps of a length-2^lg transform from sub-length 2^first_lgM down:
// radix-8 while at least 3 bits remain, then one radix-2 or radix-4 step at
// the bottom (whose twiddles are all 1).
template <bool WS = false>
__device__ __forceinline__ void fwd_steps_from(uint32_t *buf, uint32_t lg, uint32_t first_lgM, uint32_t cnt_lg,
                                               const uint32_t *__restrict__ tw, const PrimeConst &M, uint32_t tid,
                                               uint32_t nt) {
    uint32_t lgM = first_lgM;
    while (lgM >= 3) {
        if (lgM > 3)
            fwd_step<8, true, WS>(buf, lg, lgM, cnt_lg, tw, M, tid, nt);
        else
            fwd_step<8, false, WS>(buf, lg, lgM, cnt_lg, tw, M, tid, nt);
        lgM -= 3;
    }
    if (lgM == 2) fwd_step<4, false, WS>(buf, lg, 2, cnt_lg, tw, M, tid, nt);
    if (lgM == 1) fwd_step<2, false, WS>(buf, lg, 1, cnt_lg, tw, M, tid, nt);
}

// Inverse steps bottom-up, up to and including sub-length 2^last_lgM.
template <bool WS = false>
__device__ __forceinline__ void inv_steps_to(uint32_t *buf, uint32_t lg, uint32_t last_lgM, uint32_t cnt_lg,
                                             const uint32_t *__restrict__ twi, const PrimeConst &M, uint32_t tid,
                                             uint32_t nt) {
    const uint32_t r = lg % 3;
    if (r == 2) inv_step<4, false, WS>(buf, lg, 2, cnt_lg, twi, M, tid, nt);
    if (r == 1) inv_step<2, false, WS>(buf, lg, 1, cnt_lg, twi, M, tid, nt);
    for (uint32_t lgM = r + 3; lgM <= last_lgM; lgM += 3) {
        if (lgM > 3)
            inv_step<8, true, WS>(buf, lg, lgM, cnt_lg, twi, M, tid, nt);
        else
            inv_step<8, false, WS>(buf, lg, lgM, cnt_lg, twi, M, tid, nt);
    }
}

}  // namespace pa
