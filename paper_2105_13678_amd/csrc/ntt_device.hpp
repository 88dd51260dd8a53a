// Device building blocks of the number-theoretic transforms: Montgomery
// arithmetic modulo three ~31-bit primes, radix-2/4/8 butterflies and the LDS
// steps of a tile transform.
//
// Every prime p satisfies p < 2^31, so a + b < 2^32 for a, b < p, and the
// Montgomery product (R = 2^32) of any a < 2^32 with b < p is exact in 64 bits
// before its final conditional subtraction.  On gfx950 all 32x32-bit
// multiplies (v_mad_u64_u32, v_mul_lo_u32) are full-rate VALU instructions;
// a modular product costs five, an addition or subtraction three.
#pragma once

#include "pa_internal.hpp"

namespace pa {

// ---------------------------------------------------------------- field ops
// Values are canonical in [0, p).

// a * b * 2^-32 mod p, for a < 2^32 and b < p.
__device__ __forceinline__ uint32_t mmul(uint32_t a, uint32_t b, const PrimeConst &M) {
    const uint64_t t = (uint64_t)a * b;
    const uint32_t m = (uint32_t)t * M.pinv;
    const uint64_t u = (uint64_t)m * M.p + t;  // divisible by 2^32, below 2^33 p <= 2^64
    const uint32_t r = (uint32_t)(u >> 32);   // r < 2p
    return min(r, r - M.p);
}

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
// Forward (decimation in frequency): natural order in, output slot s holds
// frequency bitrev(s).  The stage with half-size h multiplies the difference
// at offset j by omega_{2h}^j = omega_16^(j*8/h) = M.w16[j*8/h].

__device__ __forceinline__ void bfly(uint32_t &u, uint32_t &v, const PrimeConst &M) {
    const uint32_t a = madd(u, v, M), b = msub(u, v, M);
    u = a;
    v = b;
}

template <int R>
__device__ __forceinline__ void dft_fwd(uint32_t *v, const PrimeConst &M) {
#pragma unroll
    for (int h = R / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int blk = 0; blk < R; blk += 2 * h) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                bfly(v[blk + j], v[blk + j + h], M);
                if (j) v[blk + j + h] = mmul(v[blk + j + h], M.w16[j * (8 / h)], M);
            }
        }
    }
}

// Forward DFT when the upper half of the input (v[R/2..R)) is known zero: the
// first stage is v[j + R/2] = v[j] * omega_R^j.
template <int R>
__device__ __forceinline__ void dft_fwd_lowhalf(uint32_t *v, const PrimeConst &M) {
    constexpr int H = R / 2;
#pragma unroll
    for (int j = 0; j < H; ++j) v[j + H] = j ? mmul(v[j], M.w16[j * (8 / H)], M) : v[j];
#pragma unroll
    for (int h = H / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int blk = 0; blk < R; blk += 2 * h) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                bfly(v[blk + j], v[blk + j + h], M);
                if (j) v[blk + j + h] = mmul(v[blk + j + h], M.w16[j * (8 / h)], M);
            }
        }
    }
}

// Inverse (times R): undoes the forward stages in reverse order with
// omega^-1 (M.w16i); bit-reversed slots in, natural order out.
template <int R>
__device__ __forceinline__ void dft_inv(uint32_t *v, const PrimeConst &M) {
#pragma unroll
    for (int h = 1; h < R; h <<= 1) {
#pragma unroll
        for (int blk = 0; blk < R; blk += 2 * h) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                if (j) v[blk + j + h] = mmul(v[blk + j + h], M.w16i[j * (8 / h)], M);
                bfly(v[blk + j], v[blk + j + h], M);
            }
        }
    }
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
// frequency): for each block b and n1 < M' = M/R, the R values
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
    uint32_t v[R];
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = buf[tile_swz(((base + ((uint32_t)j << lgMp)) << cnt_lg) + q, cnt_lg)];
    dft_fwd<R>(v, M);
    if (TW) {
#pragma unroll
        for (int s = 1; s < R; ++s) v[s] = mmul(v[s], tw[(n1 * brev_small(s, LR)) << (lg - lgM)], M);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) buf[tile_swz(((base + ((uint32_t)j << lgMp)) << cnt_lg) + q, cnt_lg)] = v[j];
}

// Inverse of fwd_task: multiply slot s by omega_M^-(n1*k2), inverse R-point
// DFT, natural order back.  twi[e] = omega_len^-e.
template <int R, bool TW>
__device__ __forceinline__ void inv_task(uint32_t *buf, uint32_t task, uint32_t lg, uint32_t lgM,
                                         uint32_t cnt_lg, const uint32_t *__restrict__ twi, const PrimeConst &M) {
    constexpr int LR = Lg<R>::v;
    const uint32_t lgMp = lgM - LR;
    const uint32_t q = task & ((1u << cnt_lg) - 1);
    const uint32_t rest = task >> cnt_lg;
    const uint32_t n1 = rest & ((1u << lgMp) - 1);
    const uint32_t base = ((rest >> lgMp) << lgM) + n1;
    uint32_t v[R];
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = buf[tile_swz(((base + ((uint32_t)j << lgMp)) << cnt_lg) + q, cnt_lg)];
    if (TW) {
#pragma unroll
        for (int s = 1; s < R; ++s) v[s] = mmul(v[s], twi[(n1 * brev_small(s, LR)) << (lg - lgM)], M);
    }
    dft_inv<R>(v, M);
#pragma unroll
    for (int j = 0; j < R; ++j) buf[tile_swz(((base + ((uint32_t)j << lgMp)) << cnt_lg) + q, cnt_lg)] = v[j];
}

template <int R, bool TW>
__device__ __forceinline__ void fwd_step(uint32_t *buf, uint32_t lg, uint32_t lgM, uint32_t cnt_lg,
                                         const uint32_t *__restrict__ tw, const PrimeConst &M, uint32_t tid,
                                         uint32_t nt) {
    const uint32_t ntask = (1u << (lg - Lg<R>::v)) << cnt_lg;
    for (uint32_t t = tid; t < ntask; t += nt) fwd_task<R, TW>(buf, t, lg, lgM, cnt_lg, tw, M);
    __syncthreads();
}

template <int R, bool TW>
__device__ __forceinline__ void inv_step(uint32_t *buf, uint32_t lg, uint32_t lgM, uint32_t cnt_lg,
                                         const uint32_t *__restrict__ twi, const PrimeConst &M, uint32_t tid,
                                         uint32_t nt) {
    const uint32_t ntask = (1u << (lg - Lg<R>::v)) << cnt_lg;
    for (uint32_t t = tid; t < ntask; t += nt) inv_task<R, TW>(buf, t, lg, lgM, cnt_lg, twi, M);
    __syncthreads();
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
__device__ __forceinline__ void fwd_steps_from(uint32_t *buf, uint32_t lg, uint32_t first_lgM, uint32_t cnt_lg,
                                               const uint32_t *__restrict__ tw, const PrimeConst &M, uint32_t tid,
                                               uint32_t nt) {
    uint32_t lgM = first_lgM;
    while (lgM >= 3) {
        if (lgM > 3)
            fwd_step<8, true>(buf, lg, lgM, cnt_lg, tw, M, tid, nt);
        else
            fwd_step<8, false>(buf, lg, lgM, cnt_lg, tw, M, tid, nt);
        lgM -= 3;
    }
    if (lgM == 2) fwd_step<4, false>(buf, lg, 2, cnt_lg, tw, M, tid, nt);
    if (lgM == 1) fwd_step<2, false>(buf, lg, 1, cnt_lg, tw, M, tid, nt);
}

// Inverse steps bottom-up, up to and including sub-length 2^last_lgM.
__device__ __forceinline__ void inv_steps_to(uint32_t *buf, uint32_t lg, uint32_t last_lgM, uint32_t cnt_lg,
                                             const uint32_t *__restrict__ twi, const PrimeConst &M, uint32_t tid,
                                             uint32_t nt) {
    const uint32_t r = lg % 3;
    if (r == 2) inv_step<4, false>(buf, lg, 2, cnt_lg, twi, M, tid, nt);
    if (r == 1) inv_step<2, false>(buf, lg, 1, cnt_lg, twi, M, tid, nt);
    for (uint32_t lgM = r + 3; lgM <= last_lgM; lgM += 3) {
        if (lgM > 3)
            inv_step<8, true>(buf, lg, lgM, cnt_lg, twi, M, tid, nt);
        else
            inv_step<8, false>(buf, lg, lgM, cnt_lg, twi, M, tid, nt);
    }
}

}  // namespace pa
