// HIP kernels of the MMH-MH hash for gfx950 (CDNA4, 64-wide wavefronts).
//
// Pipeline for one block (Algorithm 1 of arXiv 2105.13678):
//   MMH (Sec. 2.1 eq. 2): unpack key chunks x_i and seeds a_i into B-bit limbs,
//        forward NTT of all 2k limb arrays modulo each of three primes,
//        pointwise multiply-accumulate sum_i A_i * X_i in the transform
//        domain, one inverse NTT per prime, Chinese-remainder reconstruction
//        -> exact coefficients of S = sum_i a_i x_i.
//   fold (Sec. 3.1, x mod M = floor(x/2^gamma) + x mod 2^gamma): fold the
//        coefficients above bit gamma onto the low part, carry-normalise,
//        fold the small overflow back and canonicalise -> y in [0, p).
//   MH (Sec. 2.2 eq. 4): NTT product b*y, add c while carrying the low gamma
//        bits, keep bits [gamma - r, gamma) -> z.
//
// NTT of length N = N1 * N2 (four-step): a column pass does length-N1
// transforms on strided columns (LDS tile of 2^c_lg columns), a row pass does
// the four-step twiddle multiply and length-N2 transforms on contiguous rows.
// The MMH row pass transforms x_i and a_i rows, accumulates their product
// over i and immediately runs the inverse row transform on the accumulated
// row, so the transform-domain sum never goes back to HBM.  The inverse
// column pass returns natural-order residues; 1/N is folded into the inverse
// twiddles.  Every pass runs register radix-8 steps with LDS exchanges.
//
// Carry propagation uses carry transfer functions f(c) = g + [c >= th]
// (exact for the small carries that occur), composed with wavefront shuffles
// inside a workgroup and a reduce / tile-prefix / apply sequence across
// workgroups.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "ntt_device.hpp"
#include "pa_internal.hpp"
#include "pa_multi.hpp"

using namespace pa;

extern __shared__ uint32_t lds_dyn[];

namespace {

constexpr int COL_THREADS = 256;
constexpr int ROW_EPT = 16;  // row elements per thread
constexpr int ROW_MAX_THREADS = 1024;

// The transform kernels are instantiated once per hash stage (the MMH sum of
// eq. 2 and the MH product of eq. 4) so that profiles report the two stages'
// launches under separate names; the code is identical.
constexpr int STAGE_MMH = 0, STAGE_MH = 1;
constexpr unsigned MH_COL_ZSPLIT = 3;  // workgroups per tile of the MH forward column pass

__device__ __forceinline__ uint32_t bitrev(uint32_t x, uint32_t bits) {
    return bits ? (__brev(x) >> (32 - bits)) : 0u;
}

// The value of v, made opaque to the optimiser: addresses derived from it
// inside a loop are then recomputed there (one XOR or multiply each) instead
// of being hoisted out of the loop as dozens of live registers.  Emits no
// instruction.
__device__ __forceinline__ uint32_t opaque(uint32_t v) {
    asm volatile("" : "+v"(v));
    return v;
}

// The word at byte address a of an LDS array.  With a statically sized
// array its base is a compile-time constant that folds into the ds
// instruction (dynamic LDS would cost one add per access).
__device__ __forceinline__ uint32_t &lds_word(uint32_t *lds, uint32_t a) { return *(uint32_t *)((char *)lds + a); }

// Workgroup b of a G-workgroup grid is dispatched to XCD b % 8; hand each XCD
// a contiguous range of tiles so neighbouring tiles share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t G) {
    uint32_t x = b & 7u, i = b >> 3;
    uint32_t q = G >> 3, rr = G & 7u;
    return x * q + min(x, rr) + i;
}

// Position of a workgroup in the grid of the block it works for.  A
// single-block launch takes it from blockIdx / gridDim; a multi-block launch
// (one launch covering the same phase of many blocks, each with its own
// arguments and grid) maps its linear workgroup index to (block, position).
struct WG {
    uint32_t x, y, z, gx, gz;
};

__device__ __forceinline__ WG wg_self() { return WG{blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, gridDim.z}; }

// Multi-block launch (pa_multi.hpp): this workgroup's block and its position
// in that block's grid; MULTI_NONE for a padding workgroup.
__device__ __forceinline__ uint32_t wg_multi(const MultiGeo *__restrict__ geo, const uint16_t *__restrict__ owner,
                                             WG &wg) {
    uint32_t x = 0, y = 0, z = 0;
    const uint32_t i = multi_locate(geo, owner, blockIdx.x, &x, &y, &z);
    if (i != MULTI_NONE) wg = WG{x, y, z, geo[i].gx, geo[i].gz};
    return i;
}

// B (<= 32) bits of a little-endian word array starting at bit `pos`; bits at
// positions >= lim read as 0.  The array holds at least ceil(lim/64) words.
__device__ __forceinline__ uint32_t bits_at(const uint64_t *__restrict__ src, uint64_t lim,
                                            uint64_t pos, uint32_t B) {
    if (pos >= lim) return 0u;
    uint64_t wi = pos >> 6;
    uint32_t sh = (uint32_t)(pos & 63);
    uint64_t v = src[wi] >> sh;
    if (sh + B > 64 && ((wi + 1) << 6) < lim) v |= src[wi + 1] << (64 - sh);
    uint64_t rem = lim - pos;
    uint32_t w = rem < B ? (uint32_t)rem : B;
    return (uint32_t)(v & ((1ull << w) - 1));
}

// Buffer resource over `words` 32-bit words at `base`: untyped 32-bit data
// format (third descriptor dword 0x00020000 on gfx9-family parts); accesses
// past the end read 0 and are not written.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const uint32_t *base, uint32_t words) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, (int)(words * 4u), 0x00020000);
}

__device__ __forceinline__ uint32_t bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}

__device__ __forceinline__ void bstore(uint32_t v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)voff, (int)soff, 0);
}

// 64 bits of a B-bit limb array starting at bit `pos`; bits >= nbits read as 0.
__device__ __forceinline__ uint64_t limbs_get64(const uint32_t *__restrict__ limbs, uint32_t B,
                                                uint64_t nbits, uint64_t pos) {
    uint64_t v = 0;
    uint32_t got = 0;
    while (got < 64) {
        uint64_t p = pos + got;
        if (p >= nbits) break;
        uint64_t m = p / B;
        uint32_t off = (uint32_t)(p - m * B);
        uint32_t take = min(B - off, 64u - got);
        uint64_t bits = ((uint64_t)limbs[m] >> off) & ((1ull << take) - 1);
        v |= bits << got;
        got += take;
    }
    return v;
}

__device__ __forceinline__ uint32_t mulmod_slow(uint32_t a, uint32_t b, uint32_t p) {
    return (uint32_t)(((uint64_t)a * b) % p);
}

__device__ __forceinline__ uint32_t powmod_slow(uint32_t b, uint64_t e, uint32_t p) {
    uint32_t r = 1;
    while (e) {
        if (e & 1) r = mulmod_slow(r, b, p);
        b = mulmod_slow(b, b, p);
        e >>= 1;
    }
    return r;
}

// ------------------------------------------------------------------ twiddles

struct TwArgs {
    uint32_t p[NPRIMES];
    uint32_t base[NPRIMES];   // root, normal form
    uint32_t scale[NPRIMES];  // factor, normal form (already includes 2^32 for Montgomery form)
};

// A table set whose key word (in device memory) already names the wanted
// contents is not rebuilt: the table kernels return at once.  Used where the
// tables live in memory that outlasts one call (hdr == nullptr: always build).
__device__ __forceinline__ bool tw_present(const uint32_t *hdr, uint32_t want) {
    return hdr != nullptr && *(const volatile uint32_t *)hdr == want;
}

// Records the key of the table set just built (after every table kernel).
__global__ void k_tw_mark(uint32_t *hdr, uint32_t want) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *hdr = want;
}

// Every word of [dst, dst + count) set to `word` (grid-stride; a fill kernel
// rather than a memset node, so the call may also be captured in a graph).
__global__ void k_fill32(uint32_t *dst, uint64_t count, uint32_t word) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = word;
}

// dst[q*count + j] = scale_q * base_q^j mod p_q  (blockIdx.y = prime q)
__global__ void k_tw_pow(uint32_t *dst, uint64_t count, TwArgs A, const uint32_t *hdr, uint32_t want) {
    if (tw_present(hdr, want)) return;
    const uint32_t q = blockIdx.y;
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count) dst[q * count + j] = mulmod_slow(A.scale[q], powmod_slow(A.base[q], j, A.p[q]), A.p[q]);
}

// Four-step twiddles in stored row order, N = sub * 2^(m1 + m2) words per
// prime (sub = 1, or 3 for three length-2^(m1+m2) transforms side by side):
// row rho = k0 * 2^m1 + r of transform k0 holds column frequency k1 =
// bitrev(r); Wf = omega_N^(e), Wi = c * omega_N^(-e) with e = (sub*k1 + k0)*n2,
// i.e. the four-step twiddle omega_{N/sub}^(k1*n2) times the column part
// omega_N^(k0*n2) of the radix-3 twiddle omega_N^(k0*n); both scaled as given
// in the arguments (Montgomery form and 1/N folded in).
// Each thread writes TW4_RUN consecutive n2 of one row (2^m2 >= 8): the
// first power directly, the rest as successive products.
constexpr uint32_t TW4_RUN = 8;

__global__ void k_tw_four(uint32_t *Wf, uint32_t *Wi, uint32_t m1, uint32_t m2, uint32_t sub, TwArgs F, TwArgs I,
                          const uint32_t *hdr, uint32_t want) {
    if (tw_present(hdr, want)) return;
    const uint32_t q = blockIdx.y;
    const uint64_t N = (uint64_t)sub << (m1 + m2);
    const uint64_t idx0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * TW4_RUN;
    if (idx0 >= N) return;
    const uint32_t rho = (uint32_t)(idx0 >> m2);
    const uint32_t n2 = (uint32_t)(idx0 & ((1u << m2) - 1));
    const uint32_t k0 = rho >> m1, r = rho & ((1u << m1) - 1);
    const uint64_t g = (uint64_t)sub * bitrev(r, m1) + k0;  // row exponent: entry n2 is omega^(g n2)
    const uint32_t pf = F.p[q], pi = I.p[q];
    const uint32_t sf = powmod_slow(F.base[q], g, pf), si = powmod_slow(I.base[q], g, pi);
    uint32_t cf = mulmod_slow(F.scale[q], powmod_slow(sf, n2, pf), pf);
    uint32_t ci = mulmod_slow(I.scale[q], powmod_slow(si, n2, pi), pi);
    for (uint32_t j = 0; j < TW4_RUN; ++j) {
        Wf[q * N + idx0 + j] = cf;
        Wi[q * N + idx0 + j] = ci;
        cf = mulmod_slow(cf, sf, pf);
        ci = mulmod_slow(ci, si, pi);
    }
}

// Row parts of the radix-f twiddles of the lengths N = f * 2^m (f = 3, 5;
// m = m1 + m2), per prime q and transform k0 < f, indexed by the column-pass
// row r < 2^m1: forward tables n0 < (f + 1) / 2, g[n0] = omega_N^(k0 (r N2 +
// n0 N/f)) (n0 = 0: the row part of omega_N^(k0 n); n0 > 0 also carry
// omega_f^(k0 n0) for the input x_(n + n0 N/f)), then the inverse table
// omega_N^(-k0 r N2); each table NPRIMES x f x 2^m1 words, Montgomery form
// (scale of the arguments).
__global__ void k_tw_gx(uint32_t *g, uint32_t f, uint32_t m1, uint32_t m2, TwArgs F, TwArgs I, const uint32_t *hdr,
                        uint32_t want) {
    if (tw_present(hdr, want)) return;
    const uint32_t q = blockIdx.y;
    const uint32_t n1 = 1u << m1;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f * n1) return;
    const uint32_t k0 = i >> m1, r = i & (n1 - 1);
    const uint32_t nf = (f + 1) / 2;
    const size_t tab = (size_t)NPRIMES * f * n1;
    const uint64_t e = (uint64_t)k0 * ((uint64_t)r << m2);
    for (uint32_t n0 = 0; n0 < nf; ++n0) {
        const uint64_t en = (uint64_t)k0 * (((uint64_t)r << m2) + ((uint64_t)n0 << (m1 + m2)));
        g[n0 * tab + q * f * n1 + i] = mulmod_slow(F.scale[q], powmod_slow(F.base[q], en, F.p[q]), F.p[q]);
    }
    g[nf * tab + q * f * n1 + i] = mulmod_slow(I.scale[q], powmod_slow(I.base[q], e, I.p[q]), I.p[q]);
}

// Step twiddles of the 4096-point row kernel rearranged so that the lanes of
// a wave read consecutive words: [j][t] = omega_4096^(t brev4(j)) for the
// 256 threads, then [j][n1] = omega_4096^(16 n1 brev4(j)) for n1 < 16.
__global__ void k_tw_r16(const uint32_t *tw, uint32_t *dst, const uint32_t *hdr, uint32_t want) {
    if (tw_present(hdr, want)) return;
    const uint32_t q = blockIdx.y;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R16_TW) return;
    uint32_t e;
    if (i < 4096u) {
        e = (i & 255u) * brev_small(i >> 8, 4);
    } else {
        const uint32_t k = i - 4096u;
        e = 16u * (k & 15u) * brev_small(k >> 4, 4);
    }
    dst[q * R16_TW + i] = tw[q * 4096u + e];
}

// ------------------------------------------------------------------ status

// The status of a hash (Alg. 1, Sec. 3.1), taken by the first workgroup of
// the fold's reconstruction kernel: any bit >= gamma in a seed word ->
// SEED_RANGE; even b -> B_EVEN (MH needs gcd(b, 2) = 1); a key chunk none of
// whose column tiles saw a limb that is not all ones -> RELOAD.  The tile
// flags are written, 0 or 1, by every workgroup of the key-chunk column pass,
// so no flag needs clearing before a hash.
struct StatusArgs {
    const uint64_t *a, *b, *c;
    uint64_t k, W, gamma;
    const uint32_t *notones;  // k x nt flags: tile x of chunk i at i * nt + x
    uint32_t nt;
    uint32_t *status;  // status[1] written
};

__device__ void hash_status(const StatusArgs &S) {
    const uint64_t topmask = (S.gamma & 63) ? ((1ull << (S.gamma & 63)) - 1) : ~0ull;
    bool range = false, reload = false;
    for (uint64_t i = threadIdx.x; i < S.k; i += blockDim.x) range |= (S.a[i * S.W + S.W - 1] & ~topmask) != 0;
    if (threadIdx.x == 0) range |= ((S.b[S.W - 1] | S.c[S.W - 1]) & ~topmask) != 0;
    // one wavefront per chunk (the loop bounds are uniform over a wavefront)
    const uint32_t lane = threadIdx.x & 63u, nw = blockDim.x >> 6;
    for (uint64_t i = threadIdx.x >> 6; i < S.k; i += nw) {
        bool seen = false;
        for (uint32_t x = lane; x < S.nt; x += 64) seen |= S.notones[i * S.nt + x] != 0u;
        if (!__any(seen)) reload = true;
    }
    const int bad_range = __syncthreads_or(range);
    const int bad_chunk = __syncthreads_or(reload);
    if (threadIdx.x == 0) {
        uint32_t f = bad_range ? ST_SEED_RANGE : 0u;
        if ((S.b[0] & 1ull) == 0) f |= ST_B_EVEN;
        if (bad_chunk) f |= ST_RELOAD;
        S.status[1] = f;
    }
}

// After the MMH column pass: RELOAD if some chunk had only all-ones limbs.
// ------------------------------------------------------------------ NTT passes

struct ColFwdArgs {
    uint32_t *X;
    uint64_t N, L, n, gamma, k, W;
    uint32_t m1, m2, c_lg, B, s_top, mode;  // mode 0: MMH (key chunks, seed chunks); 1: MH (y, b)
    uint32_t arr0;  // source array of grid row 0 (outputs are numbered from grid row 0)
    const uint64_t *key, *a, *b;
    const uint32_t *ylimbs;
    uint32_t *notones;
    const uint32_t *tw;  // per prime: omega_{N1}^e, e < N1
    uint64_t Nsub;       // length of the power-of-two transforms (N or N/3)
    const uint32_t *g3;  // N = 3 Nsub or 5 Nsub: the row twiddle tables (k_tw_gx)
    PrimeSet P;
};

// Source of the B-bit limbs of one column-pass array, uniform over a
// workgroup.  Limb j is bits [sh0 + j*stride, +B) of the 32-bit word stream
// behind `rs` (a buffer resource over exactly the words the array touches,
// so reads past them return 0), masked to the array's first `cl` valid bits
// (relative to sh0).  Key chunks and seeds are packed bit streams
// (stride = B); the MMH output y is one limb per word (stride = 32).
struct LimbSrc {
    __amdgpu_buffer_rsrc_t rs;
    uint32_t sh0, stride, B, bmask;
    int32_t cl;
};

__device__ __forceinline__ LimbSrc limb_src(const ColFwdArgs &A, uint32_t arr) {
    LimbSrc S;
    S.B = A.B;
    S.bmask = A.B >= 32 ? ~0u : (1u << A.B) - 1u;
    S.stride = A.B;
    S.sh0 = 0;
    if (A.mode == 0 && arr < A.k) {
        const uint64_t base = (uint64_t)arr * A.gamma;
        const uint64_t lim = min(A.n, base + A.gamma);
        S.sh0 = (uint32_t)(base & 31);
        S.cl = (int32_t)(lim - base);
        S.rs = rsrc_of((const uint32_t *)A.key + (base >> 5), (uint32_t)((S.sh0 + (lim - base) + 31) >> 5));
    } else if (A.mode == 0) {
        S.cl = (int32_t)A.gamma;
        S.rs = rsrc_of((const uint32_t *)(A.a + (uint64_t)(arr - A.k) * A.W), (uint32_t)((A.gamma + 31) >> 5));
    } else if (arr == 0) {
        S.stride = 32;
        S.cl = (int32_t)(32 * A.L);
        S.rs = rsrc_of(A.ylimbs, (uint32_t)A.L);
    } else {
        S.cl = (int32_t)A.gamma;
        S.rs = rsrc_of((const uint32_t *)A.b, (uint32_t)((A.gamma + 31) >> 5));
    }
    return S;
}

// Limb j of the array (0 past its valid bits).  j * stride < 2^30 because
// j < N <= 2^25.
__device__ __forceinline__ uint32_t limb_at(const LimbSrc &S, uint32_t j) {
    const uint32_t pos = S.sh0 + j * S.stride;
    const uint32_t off = (pos >> 5) * 4u;
    const uint32_t lo = bload(S.rs, off, 0), hi = bload(S.rs, off + 4u, 0);
    uint32_t v = __builtin_amdgcn_alignbit(hi, lo, pos & 31u) & S.bmask;  // ({hi, lo} >> sh)[31:0]
    const int32_t rem = S.cl - (int32_t)(j * S.stride);
    if (rem < (int32_t)S.B) v &= rem > 0 ? (1u << rem) - 1u : 0u;
    return v;
}

// Last (twiddle-free) forward step of a column tile, LDS -> global memory:
// radix R at sub-length R; slot s of block b is row b*R + s.
template <int R>
__device__ __forceinline__ void col_last_fwd(const uint32_t *buf, uint32_t lg, uint32_t c_lg, uint32_t m2,
                                             uint64_t c0, __amdgpu_buffer_rsrc_t out, const PrimeConst &M,
                                             uint32_t tid, uint32_t nt) {
    constexpr int LR = Lg<R>::v;
    const uint32_t cmask = (1u << c_lg) - 1;
    const uint32_t ntask = (1u << (lg - LR)) << c_lg;
    for (uint32_t task = tid; task < ntask; task += nt) {
        const uint32_t q = task & cmask;
        const uint32_t row0 = (task >> c_lg) << LR;
        uint32_t v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = buf[tile_swz(((row0 + j) << c_lg) + q, c_lg)];
        dft_fwd<R>(v, M);
        const uint32_t vo = ((row0 << m2) + (uint32_t)c0 + q) << 2;
#pragma unroll
        for (int j = 0; j < R; ++j) bstore(v[j], out, vo, ((uint32_t)j << m2) << 2);
    }
}

// Tiles of 128 or 256 rows x 16 columns (compile-time shapes) finish with a
// radix-16 step on 16 consecutive rows (and the 256-row tiles start with
// one): two LDS passes instead of three.  Their LDS swizzle XORs index bits
// 8-9 into bits 4-5, so that both a step over rows 16 apart (a wave covers 4
// consecutive rows of all 16 columns) and the final step (a wave covers 4
// blocks of 16 rows) touch 64 distinct banks.
template <int LG, int CLG>
struct ColR16 {
    static constexpr bool last = CLG == 4 && (LG == 7 || LG == 8);  // last step radix 16
    static constexpr bool first = CLG == 4 && LG == 8;               // first step radix 16
};

template <int LG, int CLG>
__device__ __forceinline__ uint32_t col_swz(uint32_t i, uint32_t c_lg) {
    if constexpr (ColR16<LG, CLG>::last) return i ^ (((i >> 8) & 3u) << 4);
    else return tile_swz(i, c_lg);
}

// Last forward step of a 2^lg x 16 tile in the ColR16 layout: radix 16 on
// rows 16 b .. 16 b + 15, straight to global memory (slot s -> row 16 b + s).
template <int LG>
__device__ __forceinline__ void col_last16_fwd(const uint32_t *buf, uint32_t m2, uint64_t c0,
                                               __amdgpu_buffer_rsrc_t out, const PrimeConst &M, uint32_t tid) {
    constexpr uint32_t ntask = 1u << LG;  // (2^LG / 16 blocks) x 16 columns
    for (uint32_t task = tid; task < ntask; task += COL_THREADS) {
        const uint32_t q = task & 15u;
        const uint32_t row0 = task & ~15u;  // (task >> 4) << 4
        uint32_t v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = buf[col_swz<LG, 4>(((row0 + j) << 4) + q, 4)];
        dft_fwd<16>(v, M);
        const uint32_t vo = ((row0 << m2) + (uint32_t)c0 + q) << 2;
#pragma unroll
        for (int j = 0; j < 16; ++j) bstore(v[j], out, vo, ((uint32_t)j << m2) << 2);
    }
}

// Unpack + forward column pass.  blockIdx.y selects the array: in MMH mode
// arrays 0..k-1 are the key chunks x_i and k..2k-1 the seed chunks a_i; in
// MH mode array 0 is y and array 1 is b.  Limb j of a chunk is its bits
// [jB, jB+B); limbs j >= L are the zero padding.  A workgroup unpacks the
// limbs of its tile once (TPT first-step tasks per thread, held in
// registers) and then transforms them for each prime in turn.
// N = 2^m (MIX false): since N >= 2L - 1, every limb index >= N/2 is padding,
// so rows n1 >= N1/2 of the column tile are zero and the first radix-8 step
// unpacks only four inputs.
// N = 3 Nsub (RADIX 3): for each of the three transforms k0 of the radix-3
// split as well, whose input at n < Nsub is (x_n + omega_3^k0 x_(n+Nsub))
// omega_N^(k0 n); x_(n+2Nsub) is padding since L <= Nsub * 3/2, and
// x_(n+Nsub) only reaches rows < N1/2.  N = 5 Nsub (RADIX 5): five
// transforms, inputs (x_n + omega_5^k0 x_(n+Nsub) + omega_5^(2 k0)
// x_(n+2Nsub)) omega_N^(k0 n) (L <= Nsub * 5/2: x_(n+Nsub) reaches every row,
// x_(n+2Nsub) the rows < N1/2, higher terms are padding).  Only the row part
// omega_N^(k0 r N2) of the twiddle (n = r N2 + c) is applied here; the column
// part omega_N^(k0 c) rides on the four-step twiddle of the row pass.
// The last step writes its rows straight to global memory.
// LG, CLG (nonzero): the column length 2^m1 and tile width 2^c_lg fixed at
// compile time for the common tile shapes (shifts, masks and swizzles fold
// into constants; the tile lives in static LDS).
template <int Stage, int RADIX, int TPT, int LG, int CLG>
__device__ __forceinline__ void col_fwd_body(const ColFwdArgs &A, const WG &wg) {
    static_assert(RADIX == 1 || RADIX == 3 || RADIX == 5, "length factors 1, 3, 5");
    constexpr bool MIX = RADIX != 1;
    constexpr uint32_t NSUB = (uint32_t)RADIX;
    constexpr int FR = ColR16<LG, CLG>::first ? 16 : 8;  // radix of the first step
    constexpr int FLR = FR == 16 ? 4 : 3;
    constexpr int XR = MIX ? FR : FR / 2;                          // first-step rows of a task that hold x_n
    constexpr int XR1 = RADIX == 5 ? FR : RADIX == 3 ? FR / 2 : 1;  // ... x_(n+Nsub)
    constexpr int XR2 = RADIX == 5 ? FR / 2 : 1;                    // ... x_(n+2Nsub)
    __shared__ uint32_t Lt[LG && CLG ? 1u << (LG + CLG) : 1u];
    uint32_t *lds = LG && CLG ? Lt : lds_dyn;
    // Compile-time tiles of 16 .. 256 rows stage the first step's twiddles
    // in LDS, transform by transform: the column twiddles omega_N1^e of the
    // prime (N1 words) and, for N = 3 Nsub or 5 Nsub, the row twiddles g0 (N1
    // words), g1 (N1 words for radix 5, its rows below N1 / 2 for radix 3)
    // and for radix 5 g2 (rows below N1 / 2): LDS reads instead of a dozen or
    // more global loads per task and transform.  The next transform's tables
    // are written after the barrier that ends the current first step (no
    // thread reads them any more), and the barrier at the top of the next
    // transform publishes them.
    constexpr bool STAGE = LG >= 4 && LG <= 8 && CLG != 0;
    constexpr uint32_t N1S = STAGE ? 1u << LG : 0u;
    constexpr uint32_t G1S = RADIX == 5 ? N1S : N1S / 2;  // staged rows of g1
    __shared__ uint32_t Tg[STAGE ? (RADIX == 5 ? 3 * N1S + N1S / 2 : MIX ? N1S * 2 + N1S / 2 : N1S) : 1u];
    auto stage = [&](uint32_t it) {
        if constexpr (STAGE) {
            const uint32_t k0 = it / NPRIMES, pq = it - NPRIMES * k0;
            const uint32_t *twq = A.tw + ((uint64_t)pq << LG);
            for (uint32_t e = threadIdx.x; e < N1S; e += COL_THREADS) Tg[e] = twq[e];
            if constexpr (MIX) {
                const uint32_t *g0 = A.g3 + (((size_t)pq * RADIX + k0) << LG);
                const uint32_t *g1 = g0 + ((size_t)NPRIMES * RADIX << LG);
                for (uint32_t e = threadIdx.x; e < N1S; e += COL_THREADS) Tg[N1S + e] = g0[e];
                for (uint32_t e = threadIdx.x; e < G1S; e += COL_THREADS) Tg[2 * N1S + e] = g1[e];
                if constexpr (RADIX == 5) {
                    const uint32_t *g2 = g1 + ((size_t)NPRIMES * RADIX << LG);
                    for (uint32_t e = threadIdx.x; e < N1S / 2; e += COL_THREADS) Tg[2 * N1S + G1S + e] = g2[e];
                }
            }
        }
    };
    const uint32_t tile = xcd_tile(wg.x, wg.gx);
    const uint32_t arr = wg.y + A.arr0;
    const uint32_t c_lg = CLG ? (uint32_t)CLG : A.c_lg, lg = LG ? (uint32_t)LG : A.m1;
    const uint32_t cmask = (1u << c_lg) - 1;
    const uint64_t c0 = (uint64_t)tile << c_lg;
    const bool is_key = (A.mode == 0) && arr < A.k;
    const uint32_t full = (uint32_t)((1ull << A.B) - 1), topv = (uint32_t)((1ull << A.s_top) - 1);
    const uint32_t lgMp = lg - FLR;
    const uint32_t ntask = (1u << lgMp) << c_lg;  // at most TPT * COL_THREADS
    const uint32_t Ns = (uint32_t)A.Nsub;
    const uint32_t t = threadIdx.x;
    uint32_t x[TPT][XR], x1[TPT][XR1], x2[TPT][XR2];
    {
        const LimbSrc S = limb_src(A, arr);
        const uint32_t L = (uint32_t)A.L;
        bool not_ones = false;
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const uint32_t task = t + COL_THREADS * u;
            const uint32_t q = task & cmask, n1 = task >> c_lg;
#pragma unroll
            for (int jj = 0; jj < XR; ++jj) {
                const uint32_t j = ((n1 + ((uint32_t)jj << lgMp)) << A.m2) + (uint32_t)c0 + q;  // limb index
                x[u][jj] = task < ntask ? limb_at(S, j) : 0u;
                if (is_key && task < ntask && j < L) not_ones |= (x[u][jj] != (j == L - 1 ? topv : full));
                if constexpr (MIX) {
                    if (jj >= XR1) continue;
                    x1[u][jj] = task < ntask ? limb_at(S, j + Ns) : 0u;
                    if (is_key && task < ntask && j + Ns < L)
                        not_ones |= (x1[u][jj] != (j + Ns == L - 1 ? topv : full));
                }
                if constexpr (RADIX == 5) {
                    if (jj >= XR2) continue;
                    x2[u][jj] = task < ntask ? limb_at(S, j + 2 * Ns) : 0u;
                    if (is_key && task < ntask && j + 2 * Ns < L)
                        not_ones |= (x2[u][jj] != (j + 2 * Ns == L - 1 ? topv : full));
                }
            }
        }
        if (is_key) {  // this tile's reload flag, written whatever its value
            int any = __syncthreads_or(not_ones);
            if (t == 0 && wg.z == 0) A.notones[(uint64_t)arr * wg.gx + wg.x] = any ? 1u : 0u;
        }
    }
    // the transforms (primes x radix-3 or radix-5 branches) of this workgroup's z slice:
    // wg.gz divides NSUB * NPRIMES
    const uint32_t per_z = NSUB * NPRIMES / wg.gz;
    const uint32_t it0 = wg.z * per_z, it1 = it0 + per_z;
    if constexpr (STAGE) {
        stage(it0);
        __syncthreads();
    }
#pragma unroll 1
    for (uint32_t it = it0; it < it1; ++it) {
        const uint32_t k0 = it / NPRIMES, pq = it - NPRIMES * k0;
        const PrimeConst M = A.P.c[pq];
        const uint32_t *tw = A.tw + ((uint64_t)pq << lg);
        uint32_t *out = A.X + ((uint64_t)wg.y * NPRIMES + pq) * A.N + (uint64_t)k0 * Ns;
        const __amdgpu_buffer_rsrc_t ro = rsrc_of(out, Ns);  // this transform's Nsub words
        // row twiddles of transform k0 (k_tw_gx tables g0, g1, g2)
        const uint32_t *g0 = nullptr, *g1 = nullptr, *g2 = nullptr;
        const uint32_t *tw1 = tw;  // first-step twiddles
        if constexpr (STAGE) {
            tw1 = Tg;
            g0 = Tg + N1S;
            g1 = Tg + 2 * N1S;
            g2 = Tg + 2 * N1S + G1S;
        } else if constexpr (MIX) {
            g0 = A.g3 + (((size_t)pq * RADIX + k0) << lg);
            g1 = g0 + ((size_t)NPRIMES * RADIX << lg);
            g2 = g1 + ((size_t)NPRIMES * RADIX << lg);
        }
        if (it != it0) __syncthreads();  // the previous transform's last step has read the buffer
        const uint32_t tl = opaque(t);  // task addresses are recomputed per transform, not kept live
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const uint32_t task = tl + COL_THREADS * u;
            if (task >= ntask) continue;
            const uint32_t q = task & cmask, n1 = task >> c_lg;
            uint32_t v[FR];
            if constexpr (RADIX == 5) {
#pragma unroll
                for (int jj = 0; jj < FR; ++jj) {
                    const uint32_t row = n1 + ((uint32_t)jj << lgMp);
                    v[jj] = red2(mont(x[u][jj], g0[row], M) + mont(x1[u][jj], g1[row], M), M);  // in [0, 2p)
                    if (jj < FR / 2) v[jj] = red2(v[jj] + mont(x2[u][jj & (FR / 2 - 1)], g2[row], M), M);
                }
            } else if constexpr (MIX) {
#pragma unroll
                for (int jj = 0; jj < FR; ++jj) {
                    const uint32_t row = n1 + ((uint32_t)jj << lgMp);
                    v[jj] = jj < FR / 2
                                ? red2(mont(x[u][jj], g0[row], M) + mont(x1[u][jj & (FR / 2 - 1)], g1[row], M), M)
                                : mont(x[u][jj], g0[row], M);  // in [0, 2p)
                }
            } else {
#pragma unroll
                for (int jj = 0; jj < FR / 2; ++jj) v[jj] = mont(x[u][jj], M.one, M);  // x mod p, in [0, 2p)
            }
            if (lg > (uint32_t)FLR) {
                uint32_t w[FR];
#pragma unroll
                for (int s = 1; s < FR; ++s) w[s] = tw1[n1 * brev_small(s, FLR)];
                dft_fwd_x<FR, !MIX, true>(v, w, M);
#pragma unroll
                for (int jj = 0; jj < FR; ++jj)
                    lds[col_swz<LG, CLG>(((n1 + ((uint32_t)jj << lgMp)) << c_lg) + q, c_lg)] = v[jj];
            } else {
                dft_fwd_x<FR, !MIX, false>(v, nullptr, M);
#pragma unroll
                for (int jj = 0; jj < FR; ++jj) out[((uint64_t)jj << A.m2) + c0 + q] = v[jj];
            }
        }
        if (lg == (uint32_t)FLR) continue;  // single-step transform: written straight to global memory
        __syncthreads();
        if (it + 1 < it1) stage(it + 1);
        if constexpr (ColR16<LG, CLG>::last) {
            // 2^7 = 8 x 16 and 2^8 = 16 x 16: the rest is one radix-16 step
            col_last16_fwd<LG>(lds, A.m2, c0, ro, M, tl);
            continue;
        }
        fwd_middle_steps(lds, lg, lg - 3, c_lg, tw, M, tl, COL_THREADS);
        const uint32_t ll = last_lgM(lg);
        if (ll == 3)
            col_last_fwd<8>(lds, lg, c_lg, A.m2, c0, ro, M, tl, COL_THREADS);
        else if (ll == 2)
            col_last_fwd<4>(lds, lg, c_lg, A.m2, c0, ro, M, tl, COL_THREADS);
        else
            col_last_fwd<2>(lds, lg, c_lg, A.m2, c0, ro, M, tl, COL_THREADS);
    }
}

template <int Stage, int RADIX, int TPT, int LG = 0, int CLG = 0>
__global__ __launch_bounds__(COL_THREADS) void k_col_fwd(ColFwdArgs A) { col_fwd_body<Stage, RADIX, TPT, LG, CLG>(A, wg_self()); }

template <int Stage, int RADIX, int TPT, int LG = 0, int CLG = 0>
__global__ __launch_bounds__(COL_THREADS) void km_col_fwd(const ColFwdArgs *__restrict__ tab, const MultiGeo *__restrict__ geo,
                                     const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) col_fwd_body<Stage, RADIX, TPT, LG, CLG>(tab[i], wg);
}

// ---- 512-row column tiles (N1 = 2^9), 16 columns: compile-time shape -------
// A workgroup unpacks its tile's limbs once and transforms them for each of
// the three primes in turn (and, for N = 3 Nsub, for each of the three
// transforms of the radix-3 split: nine transforms per unpack).
// Three radix-8 steps; task index tau = t + T u (u < 1024 / T) in every step:
//   step A (sub-length 512, stride 64): q = tau & 15, n1 = tau >> 4, rows
//          n1 + 64 j; from the unpacked limbs (power-of-two N: rows >= 256
//          are padding; N = 3 Nsub: all rows carry x_n, rows < 256 also
//          x_(n+Nsub), combined with the row part of the radix-3 twiddle);
//   step B (sub-length 64, stride 8): q = tau & 15, n1 = (tau >> 4) & 7,
//          block b = tau >> 7, rows 64 b + n1 + 8 j;
//   step C (sub-length 8): q = tau & 15, block b = tau >> 4, rows 8 b + j,
//          written straight to global memory.
// LDS element (row, q) lives at tile_swz(16 row + q, 4); the swizzle is
// XOR-linear, so each task swizzles its base once and XORs constant offsets.

constexpr uint32_t C9_LG = 9, C9_CLG = 4;

__device__ __forceinline__ constexpr uint32_t swz_c9(uint32_t i) { return i ^ (((i >> 7) & 3u) << 4); }

// Threads of a 512-row forward tile: 512 (two tasks each) for the MH stage's
// power-of-two lengths, whose 3 x (one or two) arrays of tiles exceed one round
// of workgroups; 256 (four tasks each) otherwise, which measured faster there.
constexpr uint32_t c9f_threads(int stage, bool mix) { return stage == STAGE_MH && !mix ? 512u : 256u; }

template <int Stage, bool MIX>
__device__ __forceinline__ void col9_fwd_body(const ColFwdArgs &A, const WG &wg) {
    constexpr uint32_t NSUB = MIX ? 3u : 1u;
    constexpr int X0_ROWS = MIX ? 8 : 4;  // step-A rows of a task holding x_n (x_(n+Nsub): rows < 4)
    constexpr uint32_t T = c9f_threads(Stage, MIX), U = 1024u / T;  // threads, tasks per thread
    __shared__ uint32_t L9[1u << (C9_LG + C9_CLG)];  // one 512 x 16 tile
    const uint32_t tile = xcd_tile(wg.x, wg.gx);
    const uint32_t arr = wg.y + A.arr0;
    const uint64_t c0 = (uint64_t)tile << C9_CLG;
    const bool is_key = (A.mode == 0) && arr < A.k;
    const uint32_t full = (uint32_t)((1ull << A.B) - 1), topv = (uint32_t)((1ull << A.s_top) - 1);
    const uint32_t t = threadIdx.x;
    const uint32_t Ns = (uint32_t)A.Nsub;
    // the tile's limbs of the four step-A tasks, unpacked once
    uint32_t x[U][X0_ROWS], x1[U][MIX ? 4 : 1];
    {
        const LimbSrc S = limb_src(A, arr);
        const uint32_t L = (uint32_t)A.L;
        bool not_ones = false;
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t tau = t + T * u;
            const uint32_t q = tau & 15u, n1 = tau >> 4;
#pragma unroll
            for (int jj = 0; jj < X0_ROWS; ++jj) {
                const uint32_t j = ((n1 + 64u * jj) << A.m2) + (uint32_t)c0 + q;  // limb index
                x[u][jj] = limb_at(S, j);
                if (is_key && j < L) not_ones |= (x[u][jj] != (j == L - 1 ? topv : full));
                if constexpr (MIX) {
                    if (jj >= 4) continue;
                    x1[u][jj] = limb_at(S, j + Ns);
                    if (is_key && j + Ns < L) not_ones |= (x1[u][jj] != (j + Ns == L - 1 ? topv : full));
                }
            }
            if constexpr (MIX) __builtin_amdgcn_sched_barrier(0);  // 24 limb loads in flight at most
        }
        if (is_key) {  // this tile's reload flag, written whatever its value
            int any = __syncthreads_or(not_ones);
            if (t == 0 && wg.z == 0) A.notones[(uint64_t)arr * wg.gx + wg.x] = any ? 1u : 0u;
        }
    }
    // the transforms (primes x radix-3 branches) of this workgroup's z slice:
    // wg.gz divides NSUB * NPRIMES
    const uint32_t per_z = NSUB * NPRIMES / wg.gz;
    const uint32_t it0 = wg.z * per_z, it1 = it0 + per_z;
#pragma unroll 1
    for (uint32_t it = it0; it < it1; ++it) {
        const uint32_t k0 = it / NPRIMES, pq = it - NPRIMES * k0;
        const PrimeConst M = A.P.c[pq];
        const __amdgpu_buffer_rsrc_t rtw = rsrc_of(A.tw + ((uint64_t)pq << C9_LG), 1u << C9_LG);
        uint32_t *out = A.X + ((uint64_t)wg.y * NPRIMES + pq) * A.N + (uint64_t)k0 * Ns;
        const __amdgpu_buffer_rsrc_t ro = rsrc_of(out, Ns);  // this transform's Nsub words
        // radix-3 row twiddles of transform k0 (tables g0, g1 of k_tw_gx)
        __amdgpu_buffer_rsrc_t rg0 = rtw, rg1 = rtw;
        if constexpr (MIX) {
            const uint32_t *g0 = A.g3 + (((size_t)pq * 3 + k0) << C9_LG);
            rg0 = rsrc_of(g0, 1u << C9_LG);
            rg1 = rsrc_of(g0 + ((size_t)NPRIMES * 3 << C9_LG), 1u << C9_LG);
        }
        if (it != it0) __syncthreads();  // the previous transform's last step has read the buffer
        const uint32_t tl = MIX ? opaque(t) : t;  // radix-3 split: recompute the task addresses per transform
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {  // step A
            const uint32_t tau = tl + T * u;
            const uint32_t n1 = tau >> 4;
            uint32_t v[8], w[8];
            if constexpr (MIX) {
                uint32_t ga[8], gb[4];
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) ga[jj] = bload(rg0, (n1 + 64u * jj) << 2, 0);
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) gb[jj] = bload(rg1, (n1 + 64u * jj) << 2, 0);
#pragma unroll
                for (int jj = 0; jj < 8; ++jj)
                    v[jj] = jj < 4 ? red2(mont(x[u][jj], ga[jj], M) + mont(x1[u][jj & 3], gb[jj & 3], M), M)
                                   : mont(x[u][jj], ga[jj], M);  // in [0, 2p)
            } else {
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) v[jj] = mont(x[u][jj], M.one, M);  // x mod p, in [0, 2p)
            }
#pragma unroll
            for (int s = 1; s < 8; ++s) w[s] = bload(rtw, (n1 * brev_small(s, 3)) << 2, 0);
            dft_fwd_x<8, !MIX, true>(v, w, M);
            const uint32_t sb = swz_c9(tau);
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) lds_word(L9, (sb ^ (1024u * jj)) << 2) = v[jj];
        }
        __syncthreads();
        // step B's twiddles depend on (t / 16) % 8 only: loaded once, after the
        // barrier (a barrier waits for loads in flight)
        uint32_t wb[8];
        {
            const uint32_t n1 = (t >> 4) & 7u;
#pragma unroll
            for (int s = 1; s < 8; ++s) wb[s] = bload(rtw, (n1 * brev_small(s, 3)) << 5, 0);
        }
#pragma unroll 1
        for (uint32_t u = 0; u < U; ++u) {  // step B
            const uint32_t tau = t + T * u;
            const uint32_t q = tau & 15u, n1 = (tau >> 4) & 7u, b = tau >> 7;
            const uint32_t sb = swz_c9(1024u * b + 16u * n1 + q);
            uint32_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = lds_word(L9, (sb ^ swz_c9(128u * j)) << 2);
            dft_fwd_tw<8>(v, wb, M);
#pragma unroll
            for (int j = 0; j < 8; ++j) lds_word(L9, (sb ^ swz_c9(128u * j)) << 2) = v[j];
        }
        __syncthreads();
#pragma unroll 1
        for (uint32_t u = 0; u < U; ++u) {  // step C
            const uint32_t tau = t + T * u;
            const uint32_t q = tau & 15u, b = tau >> 4;
            const uint32_t sb = swz_c9(128u * b + q);
            uint32_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = lds_word(L9, (sb ^ (16u * j)) << 2);
            dft_fwd<8>(v, M);
            // buffer stores: lane offset plus a uniform row offset (no 64-bit address math)
            const uint32_t vo = (((8u * b) << A.m2) + (uint32_t)c0 + q) << 2;
#pragma unroll
            for (int j = 0; j < 8; ++j) bstore(v[j], ro, vo, ((uint32_t)j << A.m2) << 2);
        }
    }
}

template <int Stage, bool MIX>
__global__ __launch_bounds__(c9f_threads(Stage, MIX)) void k_col9_fwd(ColFwdArgs A) { col9_fwd_body<Stage, MIX>(A, wg_self()); }

template <int Stage, bool MIX>
__global__ __launch_bounds__(c9f_threads(Stage, MIX)) void km_col9_fwd(const ColFwdArgs *__restrict__ tab, const MultiGeo *__restrict__ geo,
                                     const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) col9_fwd_body<Stage, MIX>(tab[i], wg);
}

// Column pass for 1024-row tiles of 8 columns (N1 = 2^10): the 512-row
// kernel's scheme with one more row bit.  Step A: radix-8 across rows 128
// apart straight from the unpacked limbs, times omega_1024^(n1 brev(s));
// step B: radix-8 across rows 16 apart, times omega_128^(n1 brev(s)); step
// C: radix-16 on 16 consecutive rows, straight to global memory.  Output row
// 128 s_A + 16 s_B + s_C holds frequency brev3(s_A) + 8 brev3(s_B) +
// 64 brev4(s_C): natural order in, bit-reversed order out, as every column
// pass.  LDS word of (row, column) row * 8 + column, swizzled by swz_c10
// (conflict-free for the three access patterns).
constexpr uint32_t C10_LG = 10, C10_CLG = 3;
__device__ __forceinline__ constexpr uint32_t swz_c10(uint32_t i) { return i ^ (((i >> 7) & 7u) << 3); }

template <int Stage, bool MIX>
__device__ __forceinline__ void col10_fwd_body(const ColFwdArgs &A, const WG &wg) {
    constexpr uint32_t NSUB = MIX ? 3u : 1u;
    constexpr int X0_ROWS = MIX ? 8 : 4;  // step-A rows of a task holding x_n (x_(n+Nsub): rows < 4)
    __shared__ uint32_t L10[1u << (C10_LG + C10_CLG)];  // one 1024 x 8 tile
    const uint32_t tile = xcd_tile(wg.x, wg.gx);
    const uint32_t arr = wg.y + A.arr0;
    const uint64_t c0 = (uint64_t)tile << C10_CLG;
    const bool is_key = (A.mode == 0) && arr < A.k;
    const uint32_t full = (uint32_t)((1ull << A.B) - 1), topv = (uint32_t)((1ull << A.s_top) - 1);
    const uint32_t t = threadIdx.x;
    const uint32_t Ns = (uint32_t)A.Nsub;
    // the tile's limbs of the four step-A tasks, unpacked once
    uint32_t x[4][X0_ROWS], x1[4][MIX ? 4 : 1];
    {
        const LimbSrc S = limb_src(A, arr);
        const uint32_t L = (uint32_t)A.L;
        bool not_ones = false;
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const uint32_t tau = t + 256u * u;
            const uint32_t q = tau & 7u, n1 = tau >> 3;
#pragma unroll
            for (int jj = 0; jj < X0_ROWS; ++jj) {
                const uint32_t j = ((n1 + 128u * jj) << A.m2) + (uint32_t)c0 + q;  // limb index
                x[u][jj] = limb_at(S, j);
                if (is_key && j < L) not_ones |= (x[u][jj] != (j == L - 1 ? topv : full));
                if constexpr (MIX) {
                    if (jj >= 4) continue;
                    x1[u][jj] = limb_at(S, j + Ns);
                    if (is_key && j + Ns < L) not_ones |= (x1[u][jj] != (j + Ns == L - 1 ? topv : full));
                }
            }
            if constexpr (MIX) __builtin_amdgcn_sched_barrier(0);  // 24 limb loads in flight at most
        }
        if (is_key) {  // this tile's reload flag, written whatever its value
            int any = __syncthreads_or(not_ones);
            if (t == 0 && wg.z == 0) A.notones[(uint64_t)arr * wg.gx + wg.x] = any ? 1u : 0u;
        }
    }
    // the transforms (primes x radix-3 branches) of this workgroup's z slice:
    // wg.gz divides NSUB * NPRIMES
    const uint32_t per_z = NSUB * NPRIMES / wg.gz;
    const uint32_t it0 = wg.z * per_z, it1 = it0 + per_z;
#pragma unroll 1
    for (uint32_t it = it0; it < it1; ++it) {
        const uint32_t k0 = it / NPRIMES, pq = it - NPRIMES * k0;
        const PrimeConst M = A.P.c[pq];
        const __amdgpu_buffer_rsrc_t rtw = rsrc_of(A.tw + ((uint64_t)pq << C10_LG), 1u << C10_LG);
        uint32_t *out = A.X + ((uint64_t)wg.y * NPRIMES + pq) * A.N + (uint64_t)k0 * Ns;
        const __amdgpu_buffer_rsrc_t ro = rsrc_of(out, Ns);  // this transform's Nsub words
        // radix-3 row twiddles of transform k0 (tables g0, g1 of k_tw_gx)
        __amdgpu_buffer_rsrc_t rg0 = rtw, rg1 = rtw;
        if constexpr (MIX) {
            const uint32_t *g0 = A.g3 + (((size_t)pq * 3 + k0) << C10_LG);
            rg0 = rsrc_of(g0, 1u << C10_LG);
            rg1 = rsrc_of(g0 + ((size_t)NPRIMES * 3 << C10_LG), 1u << C10_LG);
        }
        if (it != it0) __syncthreads();  // the previous transform's last step has read the buffer
        const uint32_t tl = MIX ? opaque(t) : t;  // radix-3 split: recompute the task addresses per transform
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {  // step A: rows n1 + 128 j
            const uint32_t tau = tl + 256u * u;
            const uint32_t n1 = tau >> 3;
            uint32_t v[8], w[8];
            if constexpr (MIX) {
                uint32_t ga[8], gb[4];
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) ga[jj] = bload(rg0, (n1 + 128u * jj) << 2, 0);
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) gb[jj] = bload(rg1, (n1 + 128u * jj) << 2, 0);
#pragma unroll
                for (int jj = 0; jj < 8; ++jj)
                    v[jj] = jj < 4 ? red2(mont(x[u][jj], ga[jj], M) + mont(x1[u][jj & 3], gb[jj & 3], M), M)
                                   : mont(x[u][jj], ga[jj], M);  // in [0, 2p)
            } else {
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) v[jj] = mont(x[u][jj], M.one, M);  // x mod p, in [0, 2p)
            }
#pragma unroll
            for (int s = 1; s < 8; ++s) w[s] = bload(rtw, (n1 * brev_small(s, 3)) << 2, 0);
            dft_fwd_x<8, !MIX, true>(v, w, M);
            const uint32_t sb = swz_c10(tau);  // word of (row n1 + 128 s, column q): tau + 1024 s
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) lds_word(L10, (sb ^ (1024u * jj)) << 2) = v[jj];
        }
        __syncthreads();
#pragma unroll 1
        for (uint32_t u = 0; u < 4; ++u) {  // step B: rows 128 b + n1 + 16 j
            const uint32_t tau = t + 256u * u;
            const uint32_t q = tau & 7u, n1 = (tau >> 3) & 15u, b = tau >> 7;
            const uint32_t sb = swz_c10(1024u * b + 8u * n1 + q);
            uint32_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = lds_word(L10, (sb ^ swz_c10(128u * j)) << 2);
            uint32_t w[8];
#pragma unroll
            for (int s = 1; s < 8; ++s) w[s] = bload(rtw, (n1 * brev_small(s, 3)) << 5, 0);
            dft_fwd_tw<8>(v, w, M);
#pragma unroll
            for (int j = 0; j < 8; ++j) lds_word(L10, (sb ^ swz_c10(128u * j)) << 2) = v[j];
        }
        __syncthreads();
#pragma unroll 1
        for (uint32_t u = 0; u < 2; ++u) {  // step C: rows 16 b + j, to global memory
            const uint32_t tau = t + 256u * u;
            const uint32_t q = tau & 7u, b = tau >> 3;
            const uint32_t sb = swz_c10(128u * b + q);
            uint32_t v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = lds_word(L10, (sb ^ (8u * j)) << 2);
            dft_fwd<16>(v, M);
            // buffer stores: lane offset plus a uniform row offset (no 64-bit address math)
            const uint32_t vo = (((16u * b) << A.m2) + (uint32_t)c0 + q) << 2;
#pragma unroll
            for (int j = 0; j < 16; ++j) bstore(v[j], ro, vo, ((uint32_t)j << A.m2) << 2);
        }
    }
}

template <int Stage, bool MIX>
__global__ __launch_bounds__(COL_THREADS) void k_col10_fwd(ColFwdArgs A) { col10_fwd_body<Stage, MIX>(A, wg_self()); }

template <int Stage, bool MIX>
__global__ __launch_bounds__(COL_THREADS) void km_col10_fwd(const ColFwdArgs *__restrict__ tab, const MultiGeo *__restrict__ geo,
                                     const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) col10_fwd_body<Stage, MIX>(tab[i], wg);
}

struct RowArgs {
    const uint32_t *X;
    const uint32_t *A;  // seed-side transforms: pair i at A + i * pair_stride
    uint64_t N, npairs, pair_stride;  // in words
    uint32_t m2;
    uint32_t *out;
    const uint32_t *Wf, *Wi, *twf, *twi;  // per prime: four-step twiddles; omega_{N2}^+-e, e < N2
    const uint32_t *r16f, *r16i;          // per prime: step twiddles of k_row16 in thread order
    uint32_t row_group;                   // k_row: threads per pair group
    PrimeSet P;
};

// First forward step of a row straight from global memory: four-step
// twiddle on load, radix-8 DFT, step twiddles, into LDS.
template <bool WS = false>
__device__ __forceinline__ void row_first_step(const uint32_t *__restrict__ g, const uint32_t *__restrict__ w,
                                               uint32_t *buf, uint32_t lg, const uint32_t *__restrict__ tw,
                                               const PrimeConst &M, uint32_t tid, uint32_t nt) {
    const uint32_t lgMp = lg - 3;
    for (uint32_t n1 = tid; n1 < (1u << lgMp); n1 += nt) {
        uint32_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t e = n1 + ((uint32_t)j << lgMp);
            v[j] = mont(g[e], w[e], M);
        }
        if (lg > 3) {
            uint32_t t8[8];
#pragma unroll
            for (int s = 1; s < 8; ++s) t8[s] = tw[n1 * brev_small(s, 3)];
            dft_fwd_tw<8>(v, t8, M);
        } else {
            dft_fwd<8>(v, M);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) buf[swz(n1 + ((uint32_t)j << lgMp))] = v[j];
    }
    step_sync<WS>();
}

// Last inverse step of a row straight to global memory (with the inverse
// four-step twiddle, 1/N and the Montgomery correction).
__device__ __forceinline__ void row_last_inv_step(const uint32_t *buf, uint32_t *__restrict__ g,
                                                  const uint32_t *__restrict__ w, uint32_t lg,
                                                  const uint32_t *__restrict__ twi, const PrimeConst &M,
                                                  uint32_t tid, uint32_t nt) {
    const uint32_t lgMp = lg - 3;
    for (uint32_t n1 = tid; n1 < (1u << lgMp); n1 += nt) {
        uint32_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = buf[swz(n1 + ((uint32_t)j << lgMp))];
        if (lg > 3) {
            uint32_t t8[8];
#pragma unroll
            for (int s = 1; s < 8; ++s) t8[s] = twi[n1 * brev_small(s, 3)];
            dft_inv_tw<8>(v, t8, M);
        } else {
            dft_inv<8>(v, M);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t e = n1 + ((uint32_t)j << lgMp);
            g[e] = mont(v[j], w[e], M);
        }
    }
}

// Row pass: for each pair (x_i, a_i): four-step twiddle and forward transform
// of both rows, accumulate their pointwise (Montgomery) product; then the
// inverse transform of the accumulated row, inverse twiddle, store.
// blockIdx.y is the prime.  Short rows need fewer threads than a wave: the
// workgroup then runs G groups of A.row_group threads, group g taking the
// pairs i = g (mod G) with its own LDS row, and the groups' sums are added
// before the inverse transform (all threads pass the same barriers: a group
// without a pair in a round transforms a stand-in pair and discards it).
// WS: every group lies in one wavefront (A.row_group <= 64), so the steps of
// a group synchronise that wavefront only; the groups' sums meet at one
// workgroup barrier, and group 0 runs the inverse transform alone.
template <int Stage, bool WS>
__device__ __forceinline__ void row_body(const RowArgs &A, const WG &wg) {
    uint32_t *lds = lds_dyn;
    const uint32_t pq = wg.y;
    const PrimeConst M = A.P.c[pq];
    const uint32_t lg = A.m2;
    const uint32_t N2 = 1u << lg;
    const uint32_t T = blockDim.x;
    const uint32_t Tg = A.row_group, G = T / Tg;  // blockDim.x = G * Tg, Tg * ROW_EPT >= N2
    const uint32_t g = threadIdx.x / Tg, tg = threadIdx.x - g * Tg;
    uint32_t *buf = lds + g * N2;
    const uint32_t rho = xcd_tile(wg.x, wg.gx);
    const uint64_t rbase = (uint64_t)rho << lg;
    const uint32_t *wf = A.Wf + pq * A.N + rbase;
    const uint32_t *twf = A.twf + ((uint64_t)pq << lg);
    const uint32_t *twi = A.twi + ((uint64_t)pq << lg);
    uint32_t acc[ROW_EPT], xr[ROW_EPT];
#pragma unroll
    for (int q = 0; q < ROW_EPT; ++q) {
        acc[q] = 0u;
        xr[q] = 0u;
    }
    for (uint64_t i0 = 0; i0 < A.npairs; i0 += G) {
        const bool active = i0 + g < A.npairs;
        const uint64_t i = active ? i0 + g : A.npairs - 1;
        const uint32_t *xrow = A.X + i * A.pair_stride + pq * A.N + rbase;
        const uint32_t *arow = A.A + i * A.pair_stride + pq * A.N + rbase;
        row_first_step<WS>(xrow, wf, buf, lg, twf, M, tg, Tg);
        fwd_steps_from<WS>(buf, lg, lg - 3, 0, twf, M, tg, Tg);
#pragma unroll
        for (int q = 0; q < ROW_EPT; ++q) {
            uint32_t e = tg + q * Tg;
            if (e < N2) xr[q] = buf[swz(e)];
        }
        step_sync<WS>();
        row_first_step<WS>(arow, wf, buf, lg, twf, M, tg, Tg);
        fwd_steps_from<WS>(buf, lg, lg - 3, 0, twf, M, tg, Tg);
#pragma unroll
        for (int q = 0; q < ROW_EPT; ++q) {
            uint32_t e = tg + q * Tg;
            if (active && e < N2) acc[q] = red2(acc[q] + mont(xr[q], buf[swz(e)], M), M);
        }
        step_sync<WS>();
    }
#pragma unroll
    for (int q = 0; q < ROW_EPT; ++q) {
        uint32_t e = tg + q * Tg;
        if (e < N2) buf[swz(e)] = acc[q];
    }
    __syncthreads();
    if (G > 1) {  // add the groups' sums into group 0's row
        if (g == 0) {
#pragma unroll
            for (int q = 0; q < ROW_EPT; ++q) {
                uint32_t e = tg + q * Tg;
                if (e >= N2) continue;
                uint32_t v = acc[q];
                for (uint32_t h = 1; h < G; ++h) v = red2(v + lds[h * N2 + swz(e)], M);
                lds[swz(e)] = v;
            }
        }
        __syncthreads();
    }
    if constexpr (WS) {  // group 0, one wavefront
        if (threadIdx.x >= Tg) return;
        inv_steps_to<true>(lds, lg, lg - 3, 0, twi, M, threadIdx.x, Tg);
        row_last_inv_step(lds, A.out + pq * A.N + rbase, A.Wi + pq * A.N + rbase, lg, twi, M, threadIdx.x, Tg);
    } else {
        inv_steps_to(lds, lg, lg - 3, 0, twi, M, threadIdx.x, T);
        row_last_inv_step(lds, A.out + pq * A.N + rbase, A.Wi + pq * A.N + rbase, lg, twi, M, threadIdx.x, T);
    }
}

template <int Stage, bool WS>
__global__ __launch_bounds__(ROW_MAX_THREADS) void k_row(RowArgs A) { row_body<Stage, WS>(A, wg_self()); }

template <int Stage, bool WS>
__global__ __launch_bounds__(ROW_MAX_THREADS) void km_row(const RowArgs *__restrict__ tab, const MultiGeo *__restrict__ geo,
                                     const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) row_body<Stage, WS>(tab[i], wg);
}

// ---- 4096-point rows: three register radix-16 steps --------------------------
// Thread t (256 per workgroup) owns 16 values in every step:
//   step 1 (sub-length 4096, stride 256): elements t + 256 j (straight from
//          global memory, four-step twiddle on load);
//   step 2 (sub-length 256, stride 16): block t/16, offset t%16;
//   step 3 (sub-length 16): elements 16 t .. 16 t + 15 (output in registers).
// The x and a rows of a pair go through the steps together (two LDS
// buffers), and their product accumulates in registers; the inverse starts
// from those registers.  LDS layout: element i of a row at word
// i + floor(i / 16) (one pad word per 16), so each access is a per-thread
// base plus a constant (the ds instructions' immediate offset, no address
// arithmetic): step 1 at t + t/16 + 272 j, step 2 at 272 (t/16) + t%16 + 17 j,
// step 3 at 17 t + j.  Steps 2 and 3 touch 64 distinct banks per wave; step
// 1 at most two lanes per bank (three lane pairs).

constexpr int R16_THREADS = 256;
constexpr uint32_t R16_LEN = 4096;
constexpr uint32_t R16_PLEN = R16_LEN + R16_LEN / 16;  // padded row buffer, words
constexpr uint32_t R16_BA = 4 * R16_PLEN;              // byte offset of the second row buffer

template <int Stage>
__device__ __forceinline__ void row16_body(const RowArgs &A, const WG &wg) {
    __shared__ uint32_t L16[2 * R16_PLEN];
    // LDS: the x row's buffer at byte 0, the a row's at byte R16_BA; byte
    // addresses are a base (buffer plus the thread's padded offset) plus a
    // constant per element.
    const uint32_t pq = wg.y;
    const PrimeConst M = A.P.c[pq];
    const uint32_t t = threadIdx.x;
    const uint32_t rho = xcd_tile(wg.x, wg.gx);
    const uint64_t rbase = (uint64_t)rho * R16_LEN;
    const uint32_t t4 = t * 4u;  // byte offset of element t in a row
    // padded bases (bytes) of this thread's three access patterns
    const uint32_t s1b = 4u * (t + (t >> 4));                 // element t + 256 j at + 1088 j
    const uint32_t s2b = 4u * (272u * (t >> 4) + (t & 15u));  // element 256 (t/16) + t%16 + 16 j at + 68 j
    const uint32_t s3b = 68u * t;                             // element 16 t + j at + 4 j
    const uint32_t n1b = t & 15u;
    // step twiddles (step 1 omega_4096^(t k2), step 2 omega_4096^(16 n1 k2))
    // from a table in thread order, so each is one coalesced load per use
    const __amdgpu_buffer_rsrc_t rw = rsrc_of(A.Wf + pq * A.N + rbase, R16_LEN);
    const __amdgpu_buffer_rsrc_t rt = rsrc_of(A.r16f + pq * R16_TW, R16_TW);
    // the transform-domain sum: acc in [0, 2p), plus up to three raw products
    // (each below 4p^2 < 2^62) pending in 64 bits, reduced together
    uint32_t acc[16];
    uint64_t pend[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        acc[j] = 0u;
        pend[j] = 0ull;
    }
    uint32_t npend = 0;
    // the row's four-step twiddles: the same for every pair and both sides,
    // loaded once (16 registers) instead of once per pair and side
    uint32_t wv[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) wv[j] = bload(rw, t4, 1024u * j);

    for (uint64_t i = 0; i < A.npairs; ++i) {
        const uint32_t *xrow = A.X + i * A.pair_stride + pq * A.N + rbase;
        const uint32_t *arow = A.A + i * A.pair_stride + pq * A.N + rbase;
        // steps 1 and 2 for the x row (side 0) and the a row (side 1), one
        // after the other to keep the register footprint small
#pragma unroll 1
        for (int side = 0; side < 2; ++side) {
            const __amdgpu_buffer_rsrc_t rg = rsrc_of(side ? arow : xrow, R16_LEN);
            const uint32_t t4l = opaque(t4), a1 = opaque((side ? R16_BA : 0u) + s1b);
            // step 1: from global, four-step twiddle, radix-16, step twiddles.
            // All 31 loads are issued before the first use (the scheduling
            // barrier keeps the compiler from interleaving load, wait and
            // use, which would expose the memory latency 16 times).
            uint32_t v[16], w[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = bload(rg, t4l, 1024u * j);
#pragma unroll
            for (int j = 1; j < 16; ++j) w[j] = bload(rt, t4l, 1024u * j);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = mont(v[j], wv[j], M);
            dft_fwd_tw<16>(v, w, M);
#pragma unroll
            for (int j = 0; j < 16; ++j) lds_word(L16, a1 + 1088u * j) = v[j];
        }
        __syncthreads();
#pragma unroll 1
        for (int side = 0; side < 2; ++side) {
            const uint32_t a2 = opaque((side ? R16_BA : 0u) + s2b), n4l = opaque(4u * n1b);
            uint32_t v[16], w[16];
            // step 2: radix-16 on stride 16, step twiddles
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = lds_word(L16, a2 + 68u * j);
#pragma unroll
            for (int j = 1; j < 16; ++j) w[j] = bload(rt, n4l, 16384u + 64u * j);
            __builtin_amdgcn_sched_barrier(0);
            dft_fwd_tw<16>(v, w, M);
#pragma unroll
            for (int j = 0; j < 16; ++j) lds_word(L16, a2 + 68u * j) = v[j];
        }
        __syncthreads();
        // step 3: radix-16 on 16 consecutive values of each row, then multiply-accumulate
        uint32_t vx[16], va[16];
        const uint32_t a3 = opaque(s3b);
#pragma unroll
        for (int j = 0; j < 16; ++j) vx[j] = lds_word(L16, a3 + 4u * j);
        dft_fwd<16>(vx, M);
#pragma unroll
        for (int j = 0; j < 16; ++j) va[j] = lds_word(L16, R16_BA + a3 + 4u * j);
        dft_fwd<16>(va, M);
#pragma unroll
        for (int j = 0; j < 16; ++j) pend[j] += (uint64_t)vx[j] * va[j];
        if (++npend == 3 || i + 1 == A.npairs) {
            // 3 * 4p^2 + 2^32 p < 2^64, and the reduction is below 4p
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                acc[j] = red2(acc[j] + red2(redc64(pend[j], M), M), M);
                pend[j] = 0ull;
            }
            npend = 0;
        }
        __syncthreads();  // the next pair overwrites the buffers
    }

    // inverse: step 3 from the accumulators, step 2, step 1 to global
    const __amdgpu_buffer_rsrc_t rti = rsrc_of(A.r16i + pq * R16_TW, R16_TW);
    dft_inv<16>(acc, M);
#pragma unroll
    for (int j = 0; j < 16; ++j) lds_word(L16, s3b + 4u * j) = acc[j];
    __syncthreads();
    uint32_t v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = lds_word(L16, s2b + 68u * j);
    uint32_t w[16];
#pragma unroll
    for (int s = 1; s < 16; ++s) w[s] = bload(rti, 4u * n1b, 16384u + 64u * s);
    __builtin_amdgcn_sched_barrier(0);
    dft_inv_tw<16>(v, w, M);
#pragma unroll
    for (int j = 0; j < 16; ++j) lds_word(L16, s2b + 68u * j) = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = lds_word(L16, s1b + 1088u * j);
    const __amdgpu_buffer_rsrc_t ro = rsrc_of(A.out + pq * A.N + rbase, R16_LEN);
    const __amdgpu_buffer_rsrc_t rwi = rsrc_of(A.Wi + pq * A.N + rbase, R16_LEN);
#pragma unroll
    for (int s = 1; s < 16; ++s) w[s] = bload(rti, t4, 1024u * s);
#pragma unroll
    for (int j = 0; j < 16; ++j) wv[j] = bload(rwi, t4, 1024u * j);  // now the inverse four-step twiddles
    __builtin_amdgcn_sched_barrier(0);
    dft_inv_tw<16>(v, w, M);
#pragma unroll
    for (int j = 0; j < 16; ++j) bstore(mont(v[j], wv[j], M), ro, t4, 1024u * j);
}

// The MH stage's row pass multiplies one pair: the x row's spectrum stays in
// registers while the seed row goes through the same LDS buffer, so a
// workgroup holds one row buffer (17 KiB) and no 64-bit accumulators, and
// more workgroups fit on a CU.  Thread mapping, LDS layout and tables as in
// row16_body.
__device__ __forceinline__ void row16_single_body(const RowArgs &A, const WG &wg) {
    __shared__ uint32_t L16[R16_PLEN];
    const uint32_t pq = wg.y;
    const PrimeConst M = A.P.c[pq];
    const uint32_t t = threadIdx.x;
    const uint32_t rho = xcd_tile(wg.x, wg.gx);
    const uint64_t rbase = (uint64_t)rho * R16_LEN;
    const uint32_t t4 = t * 4u;
    const uint32_t s1b = 4u * (t + (t >> 4));
    const uint32_t s2b = 4u * (272u * (t >> 4) + (t & 15u));
    const uint32_t s3b = 68u * t;
    const uint32_t n1b = t & 15u;
    const __amdgpu_buffer_rsrc_t rw = rsrc_of(A.Wf + pq * A.N + rbase, R16_LEN);
    const __amdgpu_buffer_rsrc_t rt = rsrc_of(A.r16f + pq * R16_TW, R16_TW);
    uint32_t vx[16], v[16];
#pragma unroll 1
    for (int side = 0; side < 2; ++side) {
        const __amdgpu_buffer_rsrc_t rg = rsrc_of((side ? A.A : A.X) + pq * A.N + rbase, R16_LEN);
        const uint32_t t4l = opaque(t4), a1 = opaque(s1b), a2 = opaque(s2b), a3 = opaque(s3b);
        if (side) __syncthreads();  // every thread has read the x row's last step
        // step 1: from global, four-step twiddle (reloaded per side: 16
        // registers fewer), radix-16, step twiddles
        uint32_t w[16], wv[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = bload(rg, t4l, 1024u * j);
#pragma unroll
        for (int j = 0; j < 16; ++j) wv[j] = bload(rw, t4l, 1024u * j);
#pragma unroll
        for (int j = 1; j < 16; ++j) w[j] = bload(rt, t4l, 1024u * j);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = mont(v[j], wv[j], M);
        dft_fwd_tw<16>(v, w, M);
#pragma unroll
        for (int j = 0; j < 16; ++j) lds_word(L16, a1 + 1088u * j) = v[j];
        __syncthreads();
        // step 2: radix-16 on stride 16, step twiddles
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = lds_word(L16, a2 + 68u * j);
#pragma unroll
        for (int j = 1; j < 16; ++j) w[j] = bload(rt, 4u * n1b, 16384u + 64u * j);
        __builtin_amdgcn_sched_barrier(0);
        dft_fwd_tw<16>(v, w, M);
#pragma unroll
        for (int j = 0; j < 16; ++j) lds_word(L16, a2 + 68u * j) = v[j];
        __syncthreads();
        // step 3: radix-16 on 16 consecutive values (this thread's own words)
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = lds_word(L16, a3 + 4u * j);
        dft_fwd<16>(v, M);
        if (side == 0) {
#pragma unroll
            for (int j = 0; j < 16; ++j) vx[j] = v[j];
        }
    }
    // the pointwise product: both factors below 2p, the product below 4p^2,
    // its reduction below 2p
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = red2(redc64((uint64_t)vx[j] * v[j], M), M);

    // inverse: step 3 (this thread's own words), step 2, step 1 to global
    const __amdgpu_buffer_rsrc_t rti = rsrc_of(A.r16i + pq * R16_TW, R16_TW);
    dft_inv<16>(v, M);
#pragma unroll
    for (int j = 0; j < 16; ++j) lds_word(L16, s3b + 4u * j) = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = lds_word(L16, s2b + 68u * j);
    uint32_t w[16];
#pragma unroll
    for (int s = 1; s < 16; ++s) w[s] = bload(rti, 4u * n1b, 16384u + 64u * s);
    __builtin_amdgcn_sched_barrier(0);
    dft_inv_tw<16>(v, w, M);
#pragma unroll
    for (int j = 0; j < 16; ++j) lds_word(L16, s2b + 68u * j) = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = lds_word(L16, s1b + 1088u * j);
    const __amdgpu_buffer_rsrc_t ro = rsrc_of(A.out + pq * A.N + rbase, R16_LEN);
    const __amdgpu_buffer_rsrc_t rwi = rsrc_of(A.Wi + pq * A.N + rbase, R16_LEN);
    uint32_t wv[16];
#pragma unroll
    for (int s = 1; s < 16; ++s) w[s] = bload(rti, t4, 1024u * s);
#pragma unroll
    for (int j = 0; j < 16; ++j) wv[j] = bload(rwi, t4, 1024u * j);
    __builtin_amdgcn_sched_barrier(0);
    dft_inv_tw<16>(v, w, M);
#pragma unroll
    for (int j = 0; j < 16; ++j) bstore(mont(v[j], wv[j], M), ro, t4, 1024u * j);
}

// The MMH stage (k pairs) runs row16_body, the MH stage (one pair)
// row16_single_body, at up to four and six waves per SIMD.
constexpr int r16_waves(int stage) { return stage == STAGE_MH ? 6 : 4; }
template <int Stage>
__device__ __forceinline__ void row16_stage_body(const RowArgs &A, const WG &wg) {
    if constexpr (Stage == STAGE_MH)
        row16_single_body(A, wg);
    else
        row16_body<Stage>(A, wg);
}

template <int Stage>
__global__ __launch_bounds__(R16_THREADS, r16_waves(Stage)) void k_row16(RowArgs A) { row16_stage_body<Stage>(A, wg_self()); }

template <int Stage>
__global__ __launch_bounds__(R16_THREADS, r16_waves(Stage)) void km_row16(const RowArgs *__restrict__ tab, const MultiGeo *__restrict__ geo,
                                     const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) row16_stage_body<Stage>(tab[i], wg);
}

struct ColInvArgs {
    uint32_t *Cc;
    uint64_t N;
    uint32_t m1, m2, c_lg;
    const uint32_t *twi;  // per prime: omega_{N1}^-e, e < N1
    uint64_t Nsub;        // words per transform: blockIdx.z's transform starts at z * Nsub
    uint32_t row_lim;     // output rows below row_lim are stored (the rest is not needed)
    PrimeSet P;
};

// First inverse step of a column tile, global memory -> LDS: the inverse of
// the last forward step (radix R at sub-length R, no twiddles).
template <int R>
__device__ __forceinline__ void col_first_inv(const uint32_t *__restrict__ cc, uint32_t *buf, uint32_t lg,
                                              uint32_t c_lg, uint32_t m2, uint64_t c0, const PrimeConst &M,
                                              uint32_t tid, uint32_t nt) {
    constexpr int LR = Lg<R>::v;
    const uint32_t cmask = (1u << c_lg) - 1;
    const uint32_t ntask = (1u << (lg - LR)) << c_lg;
    for (uint32_t task = tid; task < ntask; task += nt) {
        const uint32_t q = task & cmask;
        const uint32_t row0 = (task >> c_lg) << LR;
        uint32_t v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = cc[((uint64_t)(row0 + j) << m2) + c0 + q];
        dft_inv<R>(v, M);
#pragma unroll
        for (int j = 0; j < R; ++j) buf[tile_swz(((row0 + j) << c_lg) + q, c_lg)] = v[j];
    }
    __syncthreads();
}

// Inverse column pass (bit-reversed rows in, natural rows out), in place:
// first step straight from global memory, last step straight back.
template <int Stage>
__device__ __forceinline__ void col_inv_body(const ColInvArgs &A, const WG &wg) {
    uint32_t *lds = lds_dyn;
    const uint32_t pq = wg.y;
    const PrimeConst M = A.P.c[pq];
    const uint32_t *twi = A.twi + ((uint64_t)pq << A.m1);
    uint32_t *cc = A.Cc + pq * A.N + wg.z * A.Nsub;
    const uint32_t tile = xcd_tile(wg.x, wg.gx);
    const uint32_t c_lg = A.c_lg, lg = A.m1;
    const uint32_t cmask = (1u << c_lg) - 1;
    const uint64_t c0 = (uint64_t)tile << c_lg;
    const uint32_t lgMp = lg - 3;
    const uint32_t ntask = (1u << lgMp) << c_lg;
    if (lg == 3) {
        for (uint32_t task = threadIdx.x; task < ntask; task += blockDim.x) {
            const uint32_t q = task & cmask;
            uint32_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = cc[((uint64_t)j << A.m2) + c0 + q];
            dft_inv<8>(v, M);
#pragma unroll
            for (int j = 0; j < 8; ++j) cc[((uint64_t)j << A.m2) + c0 + q] = canon(red2(v[j], M), M);
        }
        return;
    }
    const uint32_t ll = last_lgM(lg);
    if (ll == 3)
        col_first_inv<8>(cc, lds, lg, c_lg, A.m2, c0, M, threadIdx.x, blockDim.x);
    else if (ll == 2)
        col_first_inv<4>(cc, lds, lg, c_lg, A.m2, c0, M, threadIdx.x, blockDim.x);
    else
        col_first_inv<2>(cc, lds, lg, c_lg, A.m2, c0, M, threadIdx.x, blockDim.x);
    inv_middle_steps(lds, lg, lg - 3, c_lg, twi, M, threadIdx.x, blockDim.x);
    for (uint32_t task = threadIdx.x; task < ntask; task += blockDim.x) {
        const uint32_t q = task & cmask;
        const uint32_t n1 = task >> c_lg;
        uint32_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = lds[tile_swz(((n1 + ((uint32_t)j << lgMp)) << c_lg) + q, c_lg)];
        uint32_t w[8];
#pragma unroll
        for (int s = 1; s < 8; ++s) w[s] = twi[n1 * brev_small(s, 3)];
        dft_inv_tw<8>(v, w, M);
        // canonical residues for the Chinese-remainder step
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (n1 + ((uint32_t)j << lgMp) < A.row_lim)
                cc[((uint64_t)(n1 + ((uint32_t)j << lgMp)) << A.m2) + c0 + q] = canon(red2(v[j], M), M);
    }
}

template <int Stage>
__global__ __launch_bounds__(COL_THREADS) void k_col_inv(ColInvArgs A) { col_inv_body<Stage>(A, wg_self()); }

// Inverse column pass of 128-row (32 columns) and 256-row (16 columns) tiles
// in two LDS passes, the inverse of the forward's radix-16 schedule: radix 16
// on rows 16 b .. 16 b + 15 straight from global memory, then radix 8 (128
// rows) or 16 (256 rows) with twiddles on rows n1 + 16 j (n1 < 16) straight
// back.  256 first-step tasks per tile either way.  LDS swizzle: the block
// index's low bits (index bits 9, or 8-9) XORed into the bits above the
// column, so both steps touch 64 distinct banks per wave.
template <int LG, int CLG>
__device__ __forceinline__ uint32_t inv16_swz(uint32_t i) {
    if constexpr (CLG == 5) return i ^ (((i >> 9) & 1u) << 5);
    else return i ^ (((i >> 8) & 3u) << 4);
}

template <int Stage, int LG, int CLG>
__device__ __forceinline__ void col_inv16_body(const ColInvArgs &A, const WG &wg) {
    static_assert((LG == 7 && CLG == 5) || (LG == 8 && CLG == 4), "tile shapes of the two-pass inverse");
    constexpr int LR = LG - 4;  // last step: radix 2^LR
    constexpr int RL = 1 << LR;
    constexpr uint32_t cmask = (1u << CLG) - 1;
    __shared__ uint32_t T[1u << (LG + CLG)];
    const uint32_t pq = wg.y;
    const PrimeConst M = A.P.c[pq];
    const uint32_t *twi = A.twi + ((uint64_t)pq << LG);
    uint32_t *cc = A.Cc + pq * A.N + wg.z * A.Nsub;
    const uint32_t tile = xcd_tile(wg.x, wg.gx);
    const uint64_t c0 = (uint64_t)tile << CLG;
    for (uint32_t task = threadIdx.x; task < (1u << (LG - 4 + CLG)); task += COL_THREADS) {
        const uint32_t q = task & cmask;
        const uint32_t row0 = (task >> CLG) << 4;
        uint32_t v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = cc[((uint64_t)(row0 + j) << A.m2) + c0 + q];
        dft_inv<16>(v, M);
#pragma unroll
        for (int j = 0; j < 16; ++j) T[inv16_swz<LG, CLG>(((row0 + j) << CLG) + q)] = v[j];
    }
    __syncthreads();
    for (uint32_t task = threadIdx.x; task < (16u << CLG); task += COL_THREADS) {
        const uint32_t q = task & cmask;
        const uint32_t n1 = task >> CLG;
        uint32_t v[RL], w[RL];
#pragma unroll
        for (int j = 0; j < RL; ++j) v[j] = T[inv16_swz<LG, CLG>(((n1 + ((uint32_t)j << 4)) << CLG) + q)];
#pragma unroll
        for (int s = 1; s < RL; ++s) w[s] = twi[n1 * brev_small(s, LR)];
        dft_inv_tw<RL>(v, w, M);
        // canonical residues for the Chinese-remainder step
#pragma unroll
        for (int j = 0; j < RL; ++j) {
            const uint32_t row = n1 + ((uint32_t)j << 4);
            if (row < A.row_lim) cc[((uint64_t)row << A.m2) + c0 + q] = canon(red2(v[j], M), M);
        }
    }
}

template <int Stage, int LG, int CLG>
__global__ __launch_bounds__(COL_THREADS) void k_col_inv16(ColInvArgs A) {
    col_inv16_body<Stage, LG, CLG>(A, wg_self());
}

template <int Stage, int LG, int CLG>
__global__ __launch_bounds__(COL_THREADS) void km_col_inv16(const ColInvArgs *__restrict__ tab,
                                                          const MultiGeo *__restrict__ geo,
                                                          const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) col_inv16_body<Stage, LG, CLG>(tab[i], wg);
}

template <int Stage>
__global__ __launch_bounds__(COL_THREADS) void km_col_inv(const ColInvArgs *__restrict__ tab, const MultiGeo *__restrict__ geo,
                                     const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) col_inv_body<Stage>(tab[i], wg);
}

// ------------------------------------------------------------------ carry scan

__device__ __forceinline__ CFn cf_id() { return CFn{CF_ID, CF_INF}; }

// Carry function of one limb with digit sum t (64 bits) in base 2^B: the
// carry out is (t + c) >> B = g + [c >= 2^B - (t mod 2^B)] for the small
// carries c that occur (below 2^16); a threshold above that never fires.
__device__ __forceinline__ CFn cf_limb(uint64_t t, uint32_t B) {
    const uint64_t low = t & ((1ull << B) - 1);
    const uint64_t th = (1ull << B) - low;
    return CFn{(uint32_t)(t >> B), th > 0xFFFFull ? CF_INF : (uint32_t)th};
}

// hi o lo: first the lower run `lo`, then the higher run `hi`.
__device__ __forceinline__ CFn cf_compose(CFn lo, CFn hi) {
    if (lo.g == CF_ID) return hi;
    if (hi.g == CF_ID) return lo;
    uint32_t a = hi.g + (lo.g >= hi.th ? 1u : 0u);
    if (lo.th == CF_INF) return CFn{a, CF_INF};
    uint32_t b = hi.g + (lo.g + 1u >= hi.th ? 1u : 0u);
    if (a == b) return CFn{a, CF_INF};
    return CFn{a, lo.th};
}

__device__ __forceinline__ uint32_t cf_eval(CFn f, uint32_t c) {
    return f.g == CF_ID ? c : f.g + (c >= f.th ? 1u : 0u);
}

__device__ __forceinline__ CFn cf_shfl_up(CFn f, int d) {
    return CFn{(uint32_t)__shfl_up((int)f.g, d, 64), (uint32_t)__shfl_up((int)f.th, d, 64)};
}

__device__ __forceinline__ CFn cf_shfl_down(CFn f, int d) {
    return CFn{(uint32_t)__shfl_down((int)f.g, d, 64), (uint32_t)__shfl_down((int)f.th, d, 64)};
}

// Exclusive prefix composition of the carry functions of a wavefront's
// lanes (lane 0 first): lane l receives the composition of lanes [0, l).
__device__ __forceinline__ CFn wave_scan_excl(CFn f) {
    const int lane = threadIdx.x & 63;
    CFn w = f;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const CFn o = cf_shfl_up(w, d);
        if (lane >= d) w = cf_compose(o, w);
    }
    CFn ex = cf_shfl_up(w, 1);
    if (lane == 0) ex = cf_id();
    return ex;
}

// Block-wide ordered composition of the threads' carry functions (thread 0
// first); the result is valid in thread 0.  NT threads, multiple of 64.
template <int NT>
__device__ CFn block_reduce(CFn f) {
    __shared__ CFn wsum[NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    CFn w = f;
    // lane l composes lanes [l, l + 2d) from its own [l, l + d) and lane l + d's
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const CFn o = cf_shfl_down(w, d);
        if (lane + d < 64) w = cf_compose(w, o);
    }
    if (lane == 0) wsum[wid] = w;
    __syncthreads();
    CFn tot = cf_id();
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) tot = cf_compose(tot, wsum[i]);
    return tot;
}

// Block-wide scan of carry functions.  Returns the exclusive prefix for the
// calling thread and the block total.  NT threads, multiple of 64.
template <int NT>
__device__ void block_scan(CFn f, CFn &excl, CFn &total) {
    __shared__ CFn wsum[NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    CFn w = f;
    for (int d = 1; d < 64; d <<= 1) {
        CFn o = cf_shfl_up(w, d);
        if (lane >= d) w = cf_compose(o, w);
    }
    if (lane == 63) wsum[wid] = w;
    CFn wex = cf_shfl_up(w, 1);
    if (lane == 0) wex = cf_id();
    __syncthreads();
    CFn pre = cf_id();
    for (int i = 0; i < wid; ++i) pre = cf_compose(pre, wsum[i]);
    excl = cf_compose(pre, wex);
    CFn tot = cf_id();
    for (int i = 0; i < NT / 64; ++i) tot = cf_compose(tot, wsum[i]);
    total = tot;
    __syncthreads();
}


// Inverse column pass for 512-row tiles of 16 columns (N1 = 2^9), the mirror
// of k_col9_fwd with the same task decomposition and LDS layout: the
// sub-length-8 step straight from global memory, the sub-length-64 step, and
// the sub-length-512 step straight back to global memory as canonical
// residues.  Inverse twiddles multiply a task's inputs (fused into the first
// DIT stage).
// 512 threads, two of the tile's 1024 tasks each (task index tau = t + 512 u,
// u < 2): the launch is a single round of workgroups, so a shorter chain per
// thread finishes it sooner.
constexpr uint32_t C9I_THREADS = 512, C9I_TASKS = 1024 / C9I_THREADS;

template <int Stage>
__device__ __forceinline__ void col9_inv_body(const ColInvArgs &A, const WG &wg) {
    __shared__ uint32_t L9[1u << (C9_LG + C9_CLG)];  // one 512 x 16 tile
    const uint32_t pq = wg.y;
    const PrimeConst M = A.P.c[pq];
    const __amdgpu_buffer_rsrc_t rtw = rsrc_of(A.twi + ((uint64_t)pq << C9_LG), 1u << C9_LG);
    // this transform's Nsub words, through a buffer resource: lane offset plus
    // a uniform row offset per access
    const __amdgpu_buffer_rsrc_t rc = rsrc_of(A.Cc + pq * A.N + wg.z * A.Nsub, (uint32_t)A.Nsub);
    const uint32_t c0 = xcd_tile(wg.x, wg.gx) << C9_CLG;
    const uint32_t t = threadIdx.x;
    {
        // sub-length 8: rows 8 b + j.  The launch has few workgroups (three
        // per CU), so each thread issues the loads of both its tasks before
        // the first use: one exposed memory latency instead of two.
        uint32_t v[C9I_TASKS][8];
#pragma unroll
        for (uint32_t u = 0; u < C9I_TASKS; ++u) {
            const uint32_t tau = t + C9I_THREADS * u;
            const uint32_t q = tau & 15u, b = tau >> 4;
            const uint32_t vo = (((8u * b) << A.m2) + c0 + q) << 2;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[u][j] = bload(rc, vo, ((uint32_t)j << A.m2) << 2);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (uint32_t u = 0; u < C9I_TASKS; ++u) {
            const uint32_t tau = t + C9I_THREADS * u;
            const uint32_t q = tau & 15u, b = tau >> 4;
            dft_inv<8>(v[u], M);
            const uint32_t sb = swz_c9(128u * b + q);
#pragma unroll
            for (int j = 0; j < 8; ++j) lds_word(L9, (sb ^ (16u * j)) << 2) = v[u][j];
        }
    }
    __syncthreads();
    {
        // sub-length 64: rows 64 b + n1 + 8 j; the twiddles depend on
        // (t / 16) % 8 only, loaded once after the barrier
        uint32_t w[8];
        const uint32_t n1 = (t >> 4) & 7u;
#pragma unroll
        for (int s = 1; s < 8; ++s) w[s] = bload(rtw, (n1 * brev_small(s, 3)) << 5, 0);
#pragma unroll 1
        for (uint32_t u = 0; u < C9I_TASKS; ++u) {
            const uint32_t tau = t + C9I_THREADS * u;
            const uint32_t q = tau & 15u, b = tau >> 7;
            const uint32_t sb = swz_c9(1024u * b + 16u * n1 + q);
            uint32_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = lds_word(L9, (sb ^ swz_c9(128u * j)) << 2);
            dft_inv_tw<8>(v, w, M);
#pragma unroll
            for (int j = 0; j < 8; ++j) lds_word(L9, (sb ^ swz_c9(128u * j)) << 2) = v[j];
        }
    }
    __syncthreads();
#pragma unroll 1
    for (uint32_t u = 0; u < C9I_TASKS; ++u) {  // sub-length 512: rows n1 + 64 j, to global memory
        const uint32_t tau = t + C9I_THREADS * u;
        const uint32_t q = tau & 15u, n1 = tau >> 4;
        const uint32_t sb = swz_c9(tau);
        uint32_t v[8], w[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = lds_word(L9, (sb ^ (1024u * j)) << 2);
#pragma unroll
        for (int s = 1; s < 8; ++s) w[s] = bload(rtw, (n1 * brev_small(s, 3)) << 2, 0);
        dft_inv_tw<8>(v, w, M);
        const uint32_t vo = ((n1 << A.m2) + c0 + q) << 2;
        // canonical residues for the Chinese-remainder step
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (n1 + 64u * j < A.row_lim) bstore(canon(red2(v[j], M), M), rc, vo, ((64u * j) << A.m2) << 2);
    }
}

template <int Stage>
__global__ __launch_bounds__(C9I_THREADS) void k_col9_inv(ColInvArgs A) { col9_inv_body<Stage>(A, wg_self()); }

template <int Stage>
__global__ __launch_bounds__(C9I_THREADS) void km_col9_inv(const ColInvArgs *__restrict__ tab, const MultiGeo *__restrict__ geo,
                                     const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) col9_inv_body<Stage>(tab[i], wg);
}

// Inverse column pass for 1024-row tiles of 8 columns (N1 = 2^10), the mirror
// of k_col10_fwd: radix-16 on 16 consecutive (bit-reversed) rows straight
// from global memory, radix-8 across rows 16 apart, radix-8 across rows 128
// apart straight back to global memory as canonical residues (rows below
// row_lim).  Inverse twiddles multiply a task's inputs (fused into the first
// DIT stage).
template <int Stage>
__device__ __forceinline__ void col10_inv_body(const ColInvArgs &A, const WG &wg) {
    __shared__ uint32_t L10[1u << (C10_LG + C10_CLG)];  // one 1024 x 8 tile
    const uint32_t pq = wg.y;
    const PrimeConst M = A.P.c[pq];
    const __amdgpu_buffer_rsrc_t rtw = rsrc_of(A.twi + ((uint64_t)pq << C10_LG), 1u << C10_LG);
    // this transform's Nsub words, through a buffer resource: lane offset plus
    // a uniform row offset per access
    const __amdgpu_buffer_rsrc_t rc = rsrc_of(A.Cc + pq * A.N + wg.z * A.Nsub, (uint32_t)A.Nsub);
    const uint32_t c0 = xcd_tile(wg.x, wg.gx) << C10_CLG;
    const uint32_t t = threadIdx.x;
#pragma unroll 1
    for (uint32_t u = 0; u < 2; ++u) {  // sub-length 16: rows 16 b + j
        const uint32_t tau = t + 256u * u;
        const uint32_t q = tau & 7u, b = tau >> 3;
        const uint32_t vo = (((16u * b) << A.m2) + c0 + q) << 2;
        uint32_t v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = bload(rc, vo, ((uint32_t)j << A.m2) << 2);
        dft_inv<16>(v, M);
        const uint32_t sb = swz_c10(128u * b + q);
#pragma unroll
        for (int j = 0; j < 16; ++j) lds_word(L10, (sb ^ (8u * j)) << 2) = v[j];
    }
    __syncthreads();
#pragma unroll 1
    for (uint32_t u = 0; u < 4; ++u) {  // sub-length 128: rows 128 b + n1 + 16 j
        const uint32_t tau = t + 256u * u;
        const uint32_t q = tau & 7u, n1 = (tau >> 3) & 15u, b = tau >> 7;
        const uint32_t sb = swz_c10(1024u * b + 8u * n1 + q);
        uint32_t v[8], w[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = lds_word(L10, (sb ^ swz_c10(128u * j)) << 2);
#pragma unroll
        for (int s = 1; s < 8; ++s) w[s] = bload(rtw, (n1 * brev_small(s, 3)) << 5, 0);
        dft_inv_tw<8>(v, w, M);
#pragma unroll
        for (int j = 0; j < 8; ++j) lds_word(L10, (sb ^ swz_c10(128u * j)) << 2) = v[j];
    }
    __syncthreads();
#pragma unroll 1
    for (uint32_t u = 0; u < 4; ++u) {  // sub-length 1024: rows n1 + 128 j, to global memory
        const uint32_t tau = t + 256u * u;
        const uint32_t q = tau & 7u, n1 = tau >> 3;
        const uint32_t sb = swz_c10(tau);
        uint32_t v[8], w[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = lds_word(L10, (sb ^ (1024u * j)) << 2);
#pragma unroll
        for (int s = 1; s < 8; ++s) w[s] = bload(rtw, (n1 * brev_small(s, 3)) << 2, 0);
        dft_inv_tw<8>(v, w, M);
        const uint32_t vo = ((n1 << A.m2) + c0 + q) << 2;
        // canonical residues for the Chinese-remainder step
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (n1 + 128u * j < A.row_lim) bstore(canon(red2(v[j], M), M), rc, vo, ((128u * j) << A.m2) << 2);
    }
}

template <int Stage>
__global__ __launch_bounds__(COL_THREADS) void k_col10_inv(ColInvArgs A) { col10_inv_body<Stage>(A, wg_self()); }

template <int Stage>
__global__ __launch_bounds__(COL_THREADS) void km_col10_inv(const ColInvArgs *__restrict__ tab, const MultiGeo *__restrict__ geo,
                                     const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) col10_inv_body<Stage>(tab[i], wg);
}

// Garner's reconstruction: canonical residues r_q mod p_q of a value below
// p0 p1 p2 -> the value r0 + v1 p0 + v2 p0 p1.  With the primes of a triple
// within a factor 2 of each other (K.one_sub; all but the two longest
// power-of-two lengths' triples) a value below one prime is reduced modulo
// another by one conditional subtraction, else by a Montgomery product with
// 2^32 mod p; v2 = (r2 - r0) / (p0 p1) - v1 / p1 mod p2 takes one Montgomery
// reduction of the 64-bit sum of both products.
__device__ __forceinline__ unsigned __int128 garner(uint32_t r0, uint32_t r1, uint32_t r2, const PrimeSet &P,
                                                    const CrtConst &K) {
    const PrimeConst &M1 = P.c[1], &M2 = P.c[2];
    const bool sub = K.one_sub != 0u;  // uniform
    const uint32_t r0a = sub ? min(r0, r0 - M1.p) : mmul(r0, M1.one, M1);
    const uint32_t r0b = sub ? min(r0, r0 - M2.p) : mmul(r0, M2.one, M2);
    // v1 = (r1 - r0) / p0 mod p1
    const uint32_t v1 = mmul(msub(r1, r0a, M1), K.inv_p0_mod_p1, M1);
    const uint32_t v1b = sub ? min(v1, v1 - M2.p) : mmul(v1, M2.one, M2);
    // T < 2 p2^2 < 2^61; its reduction is below 2 p2
    const uint64_t T = (uint64_t)msub(r2, r0b, M2) * K.inv_p0p1_mod_p2 + (uint64_t)(M2.p - v1b) * K.inv_p1_mod_p2;
    const uint32_t v2 = canon(redc64(T, M2), M2);
    return (unsigned __int128)r0 + (unsigned __int128)v1 * P.c[0].p + (unsigned __int128)v2 * K.p0p1;
}

struct Crt3Args {
    const uint32_t *cc;  // 3 primes x N residues: three inverse transforms of Nsub words each
    uint32_t *c96;
    uint64_t N, Nsub, count;
    uint32_t m1, m2;
    const uint32_t *gi;  // inverse radix-3 row twiddles [q][k0][r] (third k_tw_gx table)
    PrimeSet P;
    CrtConst K;
    Mix3Const X;
    StatusArgs S;  // with S.notones set (the fold): its first workgroup writes the hash status
};

// The same reconstruction for N = 3 Nsub, fused with the inverse radix-3
// step: thread j1 < Nsub takes the residues s_k0 at j1 of the three inverse
// transforms (canonical, 1/N and the column part omega_N^(-k0 c) of the
// twiddle already applied), multiplies s_1, s_2 by the row part
// omega_N^(-k0 r N2) (j1 = r N2 + c), runs the 3-point inverse DFT and
// reconstructs the coefficients j1 + n0 Nsub (n0 < 3) below `count`.
__device__ __forceinline__ void crt3_body(const Crt3Args &A, const WG &wg) {
    const uint64_t j1 = (uint64_t)wg.x * blockDim.x + threadIdx.x;
    if (A.S.notones && wg.x == 0) hash_status(A.S);
    if (j1 >= A.Nsub || j1 >= A.count) return;
    const uint32_t r = (uint32_t)(j1 >> A.m2);
    uint32_t x[3][NPRIMES];  // [n0][prime], canonical
#pragma unroll
    for (int q = 0; q < NPRIMES; ++q) {
        const PrimeConst &M = A.P.c[q];
        const uint32_t *c = A.cc + q * A.N + j1;
        const uint32_t s0 = c[0], s1 = c[A.Nsub], s2 = c[2 * A.Nsub];
        const uint32_t *gi = A.gi + (((size_t)q * 3) << A.m1);
        const uint32_t u1 = mont(s1, gi[(1u << A.m1) + r], M);  // [0, 2p)
        const uint32_t u2 = mont(s2, gi[(2u << A.m1) + r], M);
        const uint32_t a = mont(u1 + u2, A.X.neg_half[q], M);    // -(u1 + u2)/2
        const uint32_t d = mont(u1 + M.p2 - u2, A.X.h[q], M);    // h (u1 - u2)
        x[0][q] = canon(red2(s0 + red2(u1 + u2, M), M), M);
        x[1][q] = canon(red2(s0 + red2(a + d, M), M), M);
        x[2][q] = canon(red2(s0 + red2(a + M.p2 - d, M), M), M);
    }
#pragma unroll
    for (int n0 = 0; n0 < 3; ++n0) {
        const uint64_t j = j1 + (uint64_t)n0 * A.Nsub;
        if (j >= A.count) break;
        const unsigned __int128 c = garner(x[n0][0], x[n0][1], x[n0][2], A.P, A.K);
        A.c96[j] = (uint32_t)c;
        A.c96[A.N + j] = (uint32_t)(c >> 32);
        A.c96[2 * A.N + j] = (uint32_t)(c >> 64);
    }
}

__global__ void k_crt3(Crt3Args A) { crt3_body(A, wg_self()); }

__global__ void km_crt3(const Crt3Args *__restrict__ tab, const MultiGeo *__restrict__ geo,
                                     const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) crt3_body(tab[i], wg);
}

struct Crt5Args {
    const uint32_t *cc;  // 3 primes x N residues: five inverse transforms of Nsub words each
    uint32_t *c96;
    uint64_t N, Nsub, count;
    uint32_t m1, m2;
    const uint32_t *gi;  // inverse radix-5 row twiddles [q][k0][r] (the last k_tw_gx table)
    PrimeSet P;
    CrtConst K;
    Mix5Const X;
    StatusArgs S;  // with S.notones set (the fold): its first workgroup writes the hash status
};

// The reconstruction for N = 5 Nsub, fused with the inverse radix-5 step:
// thread j1 < Nsub takes the residues s_k0 at j1 of the five inverse
// transforms (canonical, 1/N and the column part omega_N^(-k0 c) of the
// twiddle already applied), multiplies s_k0 (k0 > 0) by the row part
// omega_N^(-k0 r N2) (j1 = r N2 + c), evaluates the 5-point inverse DFT
// x_(n0) = sum_k0 u_k0 omega_5^(-k0 n0) term by term (each partial sum kept
// below 2p) and reconstructs the coefficients j1 + n0 Nsub below `count`.
__device__ __forceinline__ void crt5_body(const Crt5Args &A, const WG &wg) {
    const uint64_t j1 = (uint64_t)wg.x * blockDim.x + threadIdx.x;
    if (A.S.notones && wg.x == 0) hash_status(A.S);
    if (j1 >= A.Nsub || j1 >= A.count) return;
    const uint32_t r = (uint32_t)(j1 >> A.m2);
    uint32_t x[5][NPRIMES];  // [n0][prime], canonical
#pragma unroll
    for (int q = 0; q < NPRIMES; ++q) {
        const PrimeConst &M = A.P.c[q];
        const uint32_t *c = A.cc + q * A.N + j1;
        const uint32_t *gi = A.gi + (((size_t)q * 5) << A.m1);
        uint32_t u[5];
        u[0] = c[0];  // canonical, below p
#pragma unroll
        for (int k0 = 1; k0 < 5; ++k0) u[k0] = mont(c[(uint64_t)k0 * A.Nsub], gi[((uint32_t)k0 << A.m1) + r], M);
#pragma unroll
        for (int n0 = 0; n0 < 5; ++n0) {
            uint32_t acc = u[0];  // [0, 2p) throughout
#pragma unroll
            for (int k0 = 1; k0 < 5; ++k0) {
                const uint32_t term = n0 ? mont(u[k0], A.X.wi[q][(k0 * n0) % 5], M) : u[k0];
                acc = red2(acc + term, M);
            }
            x[n0][q] = canon(acc, M);
        }
    }
#pragma unroll
    for (int n0 = 0; n0 < 5; ++n0) {
        const uint64_t j = j1 + (uint64_t)n0 * A.Nsub;
        if (j >= A.count) break;
        const unsigned __int128 c = garner(x[n0][0], x[n0][1], x[n0][2], A.P, A.K);
        A.c96[j] = (uint32_t)c;
        A.c96[A.N + j] = (uint32_t)(c >> 32);
        A.c96[2 * A.N + j] = (uint32_t)(c >> 64);
    }
}

__global__ void k_crt5(Crt5Args A) { crt5_body(A, wg_self()); }

__global__ void km_crt5(const Crt5Args *__restrict__ tab, const MultiGeo *__restrict__ geo,
                        const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) crt5_body(tab[i], wg);
}

__device__ __forceinline__ unsigned __int128 coef(const uint32_t *__restrict__ c96, uint64_t N, uint64_t j) {
    return (unsigned __int128)c96[j] | ((unsigned __int128)c96[N + j] << 32) |
           ((unsigned __int128)c96[2 * N + j] << 64);
}

// ------------------------------------------------------------------ carry chains
// A carry normalisation runs in two launches.  The digit kernel produces the
// digit sums (one per thread) and the composed carry function of each
// CARRY_TILE-digit tile: straight from the residues for N = 2^m
// (k_digit_crt), from the reconstructed coefficient planes for N = 3 * 2^m
// (k_digit_tile after k_crt3).  The apply kernel composes the functions of
// the tiles before its own into its carry-in (and handles the top limb), then
// normalises its tile.  No workgroup waits for another.  The second fold has
// no digit kernel: the first fold's apply leaves its tile functions.
constexpr int DIG_FOLD = 0, DIG_MH = 2;
// Digit kernels: DIG_THREADS threads per CARRY_TILE-digit tile, DIG_PER_THREAD
// consecutive digits each (four 512-thread workgroups fit a CU, so every tile
// of a 2^21-point block is resident at once; with 1024 threads, two per CU,
// they ran in two rounds)
constexpr int DIG_THREADS = 512;
constexpr int DIG_PER_THREAD = CARRY_TILE / DIG_THREADS;
constexpr uint32_t WRAP_LO = 32;  // lowest limbs of y written by the first fold's extra workgroup

// The second fold's rare case, settled inside the MH digits.  The first
// fold's apply writes y' = S - c 2^(nlo B) (S = T_lo + (V mod p) unreduced,
// below 2p; nlo = min(32, L - 1); c the carry into limb nlo), the word
// c | (S's limbs below nlo all ones) << 1, and per tile whether its limbs in
// [nlo, L) are all ones.  Then y = S - w p with w = [S >= p] = (c or the low
// limbs all ones) and the upper limbs all ones (c = 1 leaves S's low limbs
// below V < 2^128, never all ones), and b y + c_seed = b y' + c_seed +
// c b 2^(nlo B) + w b (mod 2^gamma): digit m gains c b_(m - nlo) + w b_m.
struct WrapFix {
    const uint64_t *b;       // MH seed b (W words), nullptr: no correction
    const uint32_t *info;    // the word c | lo_ones << 1
    const uint32_t *tflags;  // per first-fold tile: its limbs in [nlo, L) all ones
    uint64_t ntiles;         // first-fold tiles
};

struct DigitArgs {
    const uint32_t *c96;  // product coefficients, three word planes (FOLD, MH)
    const uint64_t *cseed;  // c (MH)
    WrapFix fix;            // MH
    uint64_t *t;          // digit sums out
    CFn *agg;             // tile carry functions out
    uint64_t N, ndig, M;  // digits produced; digits in the carry chain (the rest is the top limb)
    uint64_t L, ncoef, gamma;
    uint32_t B, e, Q, Q2, s_top;
};

// Digit m of the FOLD sum T = sum_{j<L} c_j 2^(Bj) + sum_{j>=L} c_j 2^(B(j-L)+e)
// (S folded once at bit gamma; 2^gamma = 1 mod p, e = BL - gamma): the B-bit
// pieces of the coefficients that overlap digit m.
__device__ __forceinline__ uint64_t fold_digit(const DigitArgs &A, uint64_t m) {
    if (A.B == 32) {
        // the B-bit pieces are the coefficients' 32-bit word planes; the
        // folded part is shifted left by e < 32 (a funnel shift of two planes)
        uint64_t sum = 0;
#pragma unroll
        for (uint32_t q = 0; q < 3; ++q)
            if (m >= q && m - q < A.L) sum += A.c96[q * A.N + m - q];
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            if (q >= A.Q2 || m < q) continue;
            const uint64_t j = A.L + m - q;
            if (j >= A.ncoef) continue;
            const uint32_t hi = q < 3 ? A.c96[q * A.N + j] : 0u;
            const uint32_t lo = q >= 1 ? A.c96[(q - 1) * A.N + j] : 0u;
            sum += A.e ? __builtin_amdgcn_alignbit(hi, lo, 32u - A.e) : hi;
        }
        return sum;
    }
    const uint64_t mask = (1ull << A.B) - 1;
    uint64_t sum = 0;
    for (uint32_t q = 0; q < A.Q; ++q)
        if (m >= q && m - q < A.L) sum += (uint64_t)(coef(A.c96, A.N, m - q) >> (A.B * q)) & mask;
    for (uint32_t q = 0; q < A.Q2; ++q) {
        if (m >= q) {
            const uint64_t j = A.L + m - q;
            if (j < A.ncoef) sum += (uint64_t)((coef(A.c96, A.N, j) << A.e) >> (A.B * q)) & mask;
        }
    }
    return sum;
}

// MH digit m < L: the limbs of c plus the pieces of the product coefficients
// below limb L (everything at or above bit gamma is dropped, mod 2^gamma).
__device__ __forceinline__ uint64_t mh_digit(const DigitArgs &A, uint64_t m) {
    if (A.B == 32) {  // c's limb m is its 32-bit word m (bits >= gamma masked); pieces are word planes
        const uint64_t bit = 32 * m;
        uint32_t cw = bit < A.gamma ? ((const uint32_t *)A.cseed)[m] : 0u;
        if (bit + 32 > A.gamma && bit < A.gamma) cw &= (1u << (A.gamma - bit)) - 1u;
        uint64_t sum = cw;
#pragma unroll
        for (uint32_t q = 0; q < 3; ++q)
            if (m >= q) sum += A.c96[q * A.N + m - q];
        return sum;
    }
    const uint64_t mask = (1ull << A.B) - 1;
    uint64_t sum = bits_at(A.cseed, A.gamma, m * A.B, A.B);
    for (uint32_t q = 0; q < A.Q; ++q)
        if (m >= q) sum += (uint64_t)(coef(A.c96, A.N, m - q) >> (A.B * q)) & mask;
    return sum;
}

// The info word of WrapFix (0 without a correction); loaded early, used by
// wrap_fix_bits after the workgroup's own loads.
__device__ __forceinline__ uint32_t wrap_fix_info(const WrapFix &F) { return F.b ? *F.info : 0u; }

// (c, w) of WrapFix as bits 0 and 1, for the calling workgroup (uniform):
// 0 in the usual case, where the info word is 0.
__device__ uint32_t wrap_fix_bits(const WrapFix &F, uint32_t info) {
    if ((info & 3u) == 0u) return 0u;
    bool all = true;
    for (uint64_t i = threadIdx.x; i < F.ntiles; i += blockDim.x) all &= F.tflags[i] != 0u;
    const int upper = __syncthreads_and(all);
    return (info & 1u) | (upper ? 2u : 0u);
}

// The WrapFix terms of MH digit m < L.
__device__ __forceinline__ uint64_t wrap_fix_terms(const DigitArgs &A, uint32_t fx, uint64_t m) {
    uint64_t add = 0;
    const uint64_t nlo = (A.L - 1) < WRAP_LO ? (A.L - 1) : WRAP_LO;
    if ((fx & 1u) && m >= nlo) add += bits_at(A.fix.b, A.gamma, (m - nlo) * A.B, A.B);
    if (fx & 2u) add += bits_at(A.fix.b, A.gamma, m * A.B, A.B);
    return add;
}

// Digits from the coefficients' word planes (N = 3 * 2^m, after k_crt3).
// Workgroup b covers digits [b CARRY_TILE, +CARRY_TILE), DIG_PER_THREAD
// consecutive ones per thread (the digits gather from several coefficients);
// writes the digit sums and the tile's composed carry function (digits below
// M only).
template <int MODE>
__device__ __forceinline__ void digit_tile_body(const DigitArgs &A, const WG &wg) {
    const uint64_t m0 = (uint64_t)wg.x * CARRY_TILE + (uint64_t)threadIdx.x * DIG_PER_THREAD;
    uint32_t info = 0;
    if constexpr (MODE == DIG_MH) info = wrap_fix_info(A.fix);
    uint64_t d[DIG_PER_THREAD];
#pragma unroll
    for (int v = 0; v < DIG_PER_THREAD; ++v)
        d[v] = m0 + v < A.ndig ? (MODE == DIG_FOLD ? fold_digit(A, m0 + v) : mh_digit(A, m0 + v)) : 0u;
    uint32_t fx = 0;
    if constexpr (MODE == DIG_MH) fx = wrap_fix_bits(A.fix, info);
    CFn f = cf_id();
#pragma unroll
    for (int v = 0; v < DIG_PER_THREAD; ++v) {
        const uint64_t m = m0 + v;
        if (m < A.ndig) {
            if constexpr (MODE == DIG_MH) {
                if (fx) d[v] += wrap_fix_terms(A, fx, m);
            }
            A.t[m] = d[v];
            if (m < A.M) f = cf_compose(f, cf_limb(d[v], A.B));
        }
    }
    const CFn total = block_reduce<DIG_THREADS>(f);
    if (threadIdx.x == 0) A.agg[wg.x] = total;
}

template <int MODE>
__global__ __launch_bounds__(DIG_THREADS) void k_digit_tile(DigitArgs A) { digit_tile_body<MODE>(A, wg_self()); }

template <int MODE>
__global__ __launch_bounds__(DIG_THREADS) void km_digit_tile(const DigitArgs *__restrict__ tab, const MultiGeo *__restrict__ geo,
                                     const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) digit_tile_body<MODE>(tab[i], wg);
}

// The same digits straight from the convolution residues, for transform
// lengths N = 2^m (coefficients in natural order): the workgroup first
// reconstructs, with Garner's method, every coefficient its CARRY_TILE digits
// draw on into LDS (a digit takes pieces of up to DIG_HALO + 1 coefficients
// at or below its own index), then forms the digit sums from there.  Slot s
// of `lo` holds coefficient m0 - DIG_HALO + s of the range [0, L) and slot s
// of `hi` coefficient L + m0 - DIG_HALO + s of [L, 2L - 1) (FOLD only),
// zero outside those ranges; each thread then forms DIG_PER_THREAD
// consecutive digits.  In the fold, workgroup 0 also writes the hash status
// (seed ranges, b odd, the Sec. 3.1 reload rule).
constexpr int DIG_HALO = 16;  // >= pieces per coefficient - 1 (at most 12 for B >= 8)

struct DigitCrtArgs {
    DigitArgs D;
    const uint32_t *cc;  // 3 primes x N canonical residues
    PrimeSet P;
    CrtConst K;
    StatusArgs S;  // with S.notones set (the fold): its first workgroup writes the hash status
};

template <int MODE>
__device__ __forceinline__ void digit_crt_body(const DigitCrtArgs &A, const WG &wg) {
    constexpr int SPAN = CARRY_TILE + DIG_HALO;
    constexpr int HS = MODE == DIG_FOLD ? SPAN : 1;  // the high range: FOLD only
    __shared__ uint32_t lo[3][SPAN];
    __shared__ uint32_t hi[3][HS];
    const DigitArgs &D = A.D;
    const uint32_t t = threadIdx.x;
    const uint64_t m0 = (uint64_t)wg.x * CARRY_TILE;
    if constexpr (MODE == DIG_FOLD) {
        if (A.S.notones && wg.x == 0) hash_status(A.S);
    }
    uint32_t info = 0;
    if constexpr (MODE == DIG_MH) info = wrap_fix_info(D.fix);
    const uint32_t *cc = A.cc;
    for (uint32_t sl = t; sl < (uint32_t)SPAN; sl += DIG_THREADS) {
        const bool pos = m0 + sl >= (uint64_t)DIG_HALO;
        const uint64_t j = m0 + sl - DIG_HALO;  // meaningful when pos
        unsigned __int128 c = 0;
        if (pos && j < D.L) c = garner(cc[j], cc[D.N + j], cc[2 * D.N + j], A.P, A.K);
        lo[0][sl] = (uint32_t)c;
        lo[1][sl] = (uint32_t)(c >> 32);
        lo[2][sl] = (uint32_t)(c >> 64);
        if constexpr (MODE == DIG_FOLD) {
            const uint64_t jh = D.L + j;
            unsigned __int128 h = 0;
            if (pos && jh < D.ncoef) h = garner(cc[jh], cc[D.N + jh], cc[2 * D.N + jh], A.P, A.K);
            hi[0][sl] = (uint32_t)h;
            hi[1][sl] = (uint32_t)(h >> 32);
            hi[2][sl] = (uint32_t)(h >> 64);
        }
    }
    __syncthreads();
    uint32_t fx = 0;
    if constexpr (MODE == DIG_MH) fx = wrap_fix_bits(D.fix, info);
    CFn f = cf_id();
#pragma unroll
    for (int dv = 0; dv < DIG_PER_THREAD; ++dv) {
        const uint32_t tl = t * DIG_PER_THREAD + dv;  // this digit's place in the tile
        const uint64_t m = m0 + tl;
        if (m < D.ndig) {
            const uint32_t s0 = tl + DIG_HALO;  // slot of coefficient m; m - q is at s0 - q
            uint64_t d = 0;
            if (D.B == 32) {
#pragma unroll
                for (uint32_t q = 0; q < 3; ++q) d += lo[q][s0 - q];
                if constexpr (MODE == DIG_FOLD) {
                    // the folded part shifted left by e < 32: a funnel shift of two planes
#pragma unroll
                    for (uint32_t q = 0; q < 4; ++q) {
                        if (q >= D.Q2) continue;
                        const uint32_t h = q < 3 ? hi[q][s0 - q] : 0u;
                        const uint32_t l = q >= 1 ? hi[q - 1][s0 - q] : 0u;
                        d += D.e ? __builtin_amdgcn_alignbit(h, l, 32u - D.e) : h;
                    }
                } else {
                    const uint64_t bit = 32 * m;
                    uint32_t cw = bit < D.gamma ? ((const uint32_t *)D.cseed)[m] : 0u;
                    if (bit + 32 > D.gamma && bit < D.gamma) cw &= (1u << (D.gamma - bit)) - 1u;
                    d += cw;
                }
            } else {
                const uint64_t mask = (1ull << D.B) - 1;
                for (uint32_t q = 0; q < D.Q; ++q) {
                    const uint32_t sl = s0 - q;
                    const unsigned __int128 c = (unsigned __int128)lo[0][sl] | ((unsigned __int128)lo[1][sl] << 32) |
                                                ((unsigned __int128)lo[2][sl] << 64);
                    d += (uint64_t)(c >> (D.B * q)) & mask;
                }
                if constexpr (MODE == DIG_FOLD) {
                    for (uint32_t q = 0; q < D.Q2; ++q) {
                        const uint32_t sl = s0 - q;
                        const unsigned __int128 h = (unsigned __int128)hi[0][sl] | ((unsigned __int128)hi[1][sl] << 32) |
                                                    ((unsigned __int128)hi[2][sl] << 64);
                        d += (uint64_t)((h << D.e) >> (D.B * q)) & mask;
                    }
                } else {
                    d += bits_at(D.cseed, D.gamma, m * D.B, D.B);
                }
            }
            if constexpr (MODE == DIG_MH) {
                if (fx) d += wrap_fix_terms(D, fx, m);
            }
            D.t[m] = d;
            if (m < D.M) f = cf_compose(f, cf_limb(d, D.B));
        }
    }
    const CFn total = block_reduce<DIG_THREADS>(f);
    if (t == 0) D.agg[wg.x] = total;
}

template <int MODE>
__global__ __launch_bounds__(DIG_THREADS) void k_digit_crt(DigitCrtArgs A) { digit_crt_body<MODE>(A, wg_self()); }

template <int MODE>
__global__ __launch_bounds__(DIG_THREADS) void km_digit_crt(const DigitCrtArgs *__restrict__ tab, const MultiGeo *__restrict__ geo,
                                     const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) digit_crt_body<MODE>(tab[i], wg);
}

constexpr int APPLY_PLAIN = 0, APPLY_FOLD = 1, APPLY_WRAP = 2;
constexpr uint32_t WRAP_TOP = 24;    // >= digits of the folded sum at and above limb gamma / B
constexpr uint32_t EXTRA_LIMBS = 10; // >= ceil(64 / B) + 1 limbs past a tile an output word reaches

struct ScanArgs {
    const uint64_t *t;   // digit sums: M regular limbs, then the top limb at index M if has_top
    uint32_t *out;       // normalised limbs
    uint64_t M;
    uint32_t B, has_top, s_top, dual;
    uint64_t ntiles;     // ceil(M / CARRY_TILE)
    const CFn *agg;      // tile carry functions of this chain
    CFn *agg_w;          // FOLD: tile carry functions of the wrap chain, out
    uint64_t Mw;         // FOLD, WRAP: regular limbs of y (L - 1; y's top limb is index Mw)
    const uint32_t *s;   // WRAP: normalised limbs of the folded sum (M1)
    uint64_t gamma, M1;  // FOLD, WRAP
    uint32_t qv;         // FOLD, WRAP: wrap digits below qv = ceil(128 / B) take pieces of V mod p
    uint32_t *y;         // FOLD: the limbs of y (usual case of the second fold)
    uint32_t *flag;      // FOLD: 1 when the usual case does not apply, else 0; WRAP: runs only on 1
    uint32_t *wrapinfo;  // FOLD: c | (low limbs of S all ones) << 1 (see WrapFix), 0 without inline wrap
    uint32_t *tflags;    // FOLD: per tile, 1 when its limbs in [nlo, L) are all ones (top limb: s_top bits)
    uint64_t *zout;      // PLAIN: if set, z = bits [gamma - r, gamma) of the result, packed
    uint64_t out_words, r;
    const uint32_t *status;  // PLAIN with zout: final status flags at index 1 (no output unless 0)
    uint32_t *dst;           // PLAIN with zout: the final flags are copied here
};

// V mod p for V < 2^128 and p = 2^gamma - 1 (identity for gamma >= 128).
__device__ __forceinline__ unsigned __int128 mod_mersenne128(unsigned __int128 V, uint64_t gamma) {
    if (gamma < 128) {
        const unsigned __int128 pm = (((unsigned __int128)1) << gamma) - 1;
        while (V >> gamma) V = (V & pm) + (V >> gamma);
        if (V == pm) V = 0;
    }
    return V;
}

// The second fold (Sec. 3.1): with the folded sum normalised into limbs s
// (M1 of them), T = T_lo + 2^gamma V with T_lo = T mod 2^gamma and V < 2^92;
// returns V mod p (p = 2^gamma - 1), which the wrap chain adds to T_lo.
__device__ __forceinline__ unsigned __int128 wrap_value(const uint32_t *__restrict__ s, uint64_t gamma, uint32_t B,
                                                        uint64_t M1) {
    unsigned __int128 V = 0;
    for (uint64_t idx = gamma / B; idx < M1; ++idx) {
        const uint64_t lo_bit = idx * B;
        const unsigned __int128 limb = s[idx];
        if (lo_bit < gamma) V += limb >> (gamma - lo_bit);
        else if (lo_bit - gamma < 128) V += limb << (lo_bit - gamma);  // higher limbs are zero
    }
    return mod_mersenne128(V, gamma);
}

// The second fold's usual case, run by one extra workgroup of the first
// fold's apply beside the tiles (no workgroup waits for another): it
// evaluates the first fold's carry chain itself at the limbs above bit gamma
// (the tiles' functions below the tile of limb gamma / B, then that tile's
// digits up to it) to get V mod p, normalises the lowest WRAP_LO digits
// (the chain's carry-in is 0), adds V's pieces to the lowest qv of them and
// lets the carry run.  y = T_lo + V then differs from T_lo only below the
// limb where the carry stops; it is canonical (below p) when some limb above
// that one, still below WRAP_LO, is not all ones: then no carry reaches bit
// gamma and not every bit of y is one.  In that case this workgroup writes
// y's lowest limbs (the tiles write the rest) and clears the flag; otherwise
// it sets the flag and the general wrap chain recomputes y.
__device__ void wrap_usual_case(const ScanArgs &A) {
    __shared__ uint64_t tlo[WRAP_LO], ttop[WRAP_TOP];
    const uint32_t t = threadIdx.x;
    const uint64_t d0 = A.gamma / A.B, T = d0 / CARRY_TILE, nv = A.M - d0;
    // every global load of the job first (one round trip to memory): the
    // lowest and the top digits, this thread's digits of tile T below d0,
    // its first aggregates of the tiles below T
    const uint64_t lo_d = t < WRAP_LO && t < A.M ? A.t[t] : 0ull;
    const uint64_t top_d = t < nv ? A.t[d0 + t] : 0ull;
    const uint64_t base = T * CARRY_TILE + (uint64_t)t * CARRY_PER_THREAD;
    uint64_t dv[CARRY_PER_THREAD];
#pragma unroll
    for (int v = 0; v < CARRY_PER_THREAD; ++v) dv[v] = base + v < d0 ? A.t[base + v] : 0ull;
    const uint64_t per = (T + SCAN_THREADS - 1) / SCAN_THREADS;
    const uint64_t j0 = min((uint64_t)t * per, T), j1 = min(j0 + per, T);
    constexpr int PRE = 8;
    CFn pre[PRE];
#pragma unroll
    for (int q = 0; q < PRE; ++q) pre[q] = j0 + q < j1 ? A.agg[j0 + q] : cf_id();
    CFn f = cf_id();
#pragma unroll
    for (int q = 0; q < PRE; ++q) f = cf_compose(f, pre[q]);
    for (uint64_t j = j0 + PRE; j < j1; ++j) f = cf_compose(f, A.agg[j]);  // beyond 8 tiles per thread
    if (t < WRAP_LO) tlo[t] = lo_d;
    if (t < nv) ttop[t] = top_d;
    const CFn below = block_reduce<SCAN_THREADS>(f);
    __syncthreads();
    CFn g = cf_id();
#pragma unroll
    for (int v = 0; v < CARRY_PER_THREAD; ++v)
        if (base + v < d0) g = cf_compose(g, cf_limb(dv[v], A.B));
    const CFn within = block_reduce<SCAN_THREADS>(g);
    __syncthreads();
    __shared__ uint64_t vw[2];  // V mod p, broadcast to wave 0
    const uint64_t mask = (1ull << A.B) - 1;
    if (t == 0) {  // V from the top digits (at most WRAP_TOP, one after another)
        uint32_t c = cf_eval(cf_compose(below, within), 0u);
        unsigned __int128 V = 0;
        for (uint64_t i = 0; i < nv; ++i) {
            const uint64_t v = ttop[i] + c;
            const unsigned __int128 limb = v & mask;
            c = (uint32_t)(v >> A.B);
            const uint64_t lo_bit = (d0 + i) * A.B;
            if (lo_bit < A.gamma) V += limb >> (A.gamma - lo_bit);
            else if (lo_bit - A.gamma < 128) V += limb << (lo_bit - A.gamma);
        }
        V = mod_mersenne128(V, A.gamma);
        vw[0] = (uint64_t)V;
        vw[1] = (uint64_t)(V >> 64);
    }
    __syncthreads();
    if (t >= 64) return;
    // wave 0, lane m < nlo: limb m of T_lo (the first fold's chain from
    // carry-in 0), then y = T_lo + V on the lowest limbs: two carry chains as
    // lane prefix compositions of the digits' carry functions
    const uint32_t nlo = (uint32_t)min((uint64_t)WRAP_LO, A.Mw);
    const bool on = t < nlo;
    const unsigned __int128 V = (unsigned __int128)vw[0] | ((unsigned __int128)vw[1] << 64);
    const uint64_t d = on ? tlo[t] : 0ull;
    const uint32_t c1 = cf_eval(wave_scan_excl(on ? cf_limb(d, A.B) : cf_id()), 0u);
    const uint64_t sl = (d + c1) & mask;  // limb t of T_lo
    const uint64_t e = sl + (on && t < A.qv ? (uint64_t)(V >> (A.B * t)) & mask : 0ull);
    const uint32_t c2 = cf_eval(wave_scan_excl(on ? cf_limb(e, A.B) : cf_id()), 0u);
    const uint64_t ys = e + c2;  // limb t of y and its carry out
    // the carry stops at the first limb m >= qv - 1 with no carry out; y's
    // limbs above it are T_lo's
    const uint64_t stop = __ballot(on && t + 1 >= A.qv && (ys >> A.B) == 0);
    const uint32_t first_same = stop ? (uint32_t)__ffsll((unsigned long long)stop) : nlo + 1;  // limb index + 1
    const uint64_t guard = __ballot(on && t >= first_same && sl != mask);
    const bool usual = A.qv < nlo && first_same <= nlo && guard != 0;
    if (A.qv < nlo) {
        // y's lowest limbs are those of S = T_lo + (V mod p) whatever the case:
        // with the tiles' limbs above them, y' = S - c 2^(nlo B) (c the carry
        // into limb nlo), which the MH digits correct (WrapFix) unless c = 0
        // and the low limbs are not all ones (then y' = y)
        if (on) A.y[t] = (uint32_t)(ys & mask);
        const uint32_t c = (uint32_t)__shfl((int)(uint32_t)(ys >> A.B), (int)nlo - 1, 64);
        const uint64_t ones = __ballot(on && (ys & mask) == mask);
        const bool lo_ones = ones == (nlo >= 64 ? ~0ull : (1ull << nlo) - 1);
        if (t == 0) *A.wrapinfo = c | (lo_ones ? 2u : 0u);
    } else if (t == 0) {
        *A.wrapinfo = 0u;
    }
    if (t == 0) *A.flag = usual ? 0u : 1u;
}

// Normalise one tile.  The carry into the tile is the composition of the
// aggregates of all earlier tiles evaluated at the chain's carry-in (every
// workgroup composes them itself: a few per thread, no second pass).  With a
// top limb (index M, s_top bits) the whole chain is also evaluated for
// carry-in 0 and 1; in dual mode the chain takes carry-in 1 when carry-in 1
// leaves a nonzero value above the top limb's width, i.e. when the sum is at
// least p (see launch_fold), and workgroup 0 writes the top limb.  Launched
// with max(1, ntiles) workgroups (FOLD: one more, see below).
//
// APPLY_FOLD also composes, per tile, the carry functions of the limbs it
// writes as digits of the wrap chain (digits [qv, Mw) only), into agg_w,
// writes its limbs from WRAP_LO up as y's limbs (y's top limb cut to s_top
// bits), and its extra workgroup (index 0; tile b runs in workgroup b + 1)
// runs the second fold's usual case.  APPLY_WRAP, which runs only when the flag says the usual case does
// not apply, runs the general wrap chain: its digits are read from the limbs
// s of the folded sum, the lowest qv with the pieces of V mod p added and
// the top one cut to s_top bits; the carry functions of digits [0, qv),
// which depend on V, are composed here (thread 0 prepends them to the
// aggregates).
// APPLY_PLAIN with zout also packs the output z (Alg. 1: the top r of the
// gamma bits): each workgroup places its limbs and the next EXTRA_LIMBS
// (normalised from the tile's carry out) in LDS and writes the output words
// that start in its limbs (the last workgroup: up to bit gamma), unless the
// status flags are set; workgroup 0 copies the flags to dst.
template <int AM>
__device__ __forceinline__ void apply_tile(const ScanArgs &A, uint64_t b, unsigned __int128 W);

template <int AM>
__device__ __forceinline__ void carry_apply_body(const ScanArgs &A, const WG &wg) {
    if constexpr (AM == APPLY_WRAP) {
        if (*(const volatile uint32_t *)A.flag == 0u) return;
        // the general case is rare: a small grid (its early exit is then
        // cheap), each workgroup taking tiles wg.x, wg.x + gx, ...
        const unsigned __int128 W = wrap_value(A.s, A.gamma, A.B, A.M1);
        const uint64_t nb = A.ntiles ? A.ntiles : 1;
        for (uint64_t b = wg.x; b < nb; b += wg.gx) {
            apply_tile<AM>(A, b, W);
            __syncthreads();  // the next tile reuses the scans' LDS
        }
        return;
    }
    if constexpr (AM == APPLY_FOLD) {
        if (wg.x == 0) {  // dispatched first: its chain of loads and reductions overlaps the tiles
            wrap_usual_case(A);
            return;
        }
    }
    apply_tile<AM>(A, AM == APPLY_FOLD ? wg.x - 1 : wg.x, 0);
}

// Tile b of an apply launch (W: V mod p of the wrap chain, APPLY_WRAP only).
template <int AM>
__device__ __forceinline__ void apply_tile(const ScanArgs &A, uint64_t b, unsigned __int128 W) {
    const uint64_t mask = (1ull << A.B) - 1;
    constexpr bool EXTRACT = AM == APPLY_PLAIN;
    __shared__ uint32_t lb[EXTRACT ? CARRY_TILE + EXTRA_LIMBS : 1];
    __shared__ uint64_t tx[EXTRACT ? EXTRA_LIMBS : 1];
    __shared__ uint32_t cout;
    const uint64_t tile_end = min((b + 1) * CARRY_TILE, A.M);
    const uint64_t tile_len = b < A.ntiles ? tile_end - b * CARRY_TILE : 0;
    if (EXTRACT && A.zout && threadIdx.x < EXTRA_LIMBS) {
        const uint64_t m = (b < A.ntiles ? tile_end : 0) + threadIdx.x;
        tx[threadIdx.x] = (m < A.M || (A.has_top && m == A.M)) ? A.t[m] : 0ull;
    }
    // the tile's digit sums (WRAP: limbs) first: their loads overlap the
    // composition below
    const uint64_t base = b * CARRY_TILE + (uint64_t)threadIdx.x * CARRY_PER_THREAD;
    uint64_t tv[CARRY_PER_THREAD];
#pragma unroll
    for (int v = 0; v < CARRY_PER_THREAD; ++v)
        tv[v] = base + v < A.M ? (AM == APPLY_WRAP ? (uint64_t)A.s[base + v] : A.t[base + v]) : 0ull;
    if constexpr (AM == APPLY_WRAP) {
#pragma unroll
        for (int v = 0; v < CARRY_PER_THREAD; ++v)
            if (base + v < A.qv && base + v < A.M) tv[v] += (uint64_t)(W >> (A.B * (base + v))) & mask;
    }
    auto digit = [&](uint64_t m) -> uint64_t {  // m <= M
        if constexpr (AM == APPLY_WRAP) {
            uint64_t d = m < A.M ? A.s[m] : (A.s[m] & ((1ull << A.s_top) - 1));
            if (m < A.qv) d += (uint64_t)(W >> (A.B * m)) & mask;
            return d;
        } else {
            return A.t[m];
        }
    };
    // aggregates of the tiles before this one (and, with a top limb, of all)
    const uint64_t per = (A.ntiles + SCAN_THREADS - 1) / SCAN_THREADS;
    const uint64_t jn = A.has_top ? A.ntiles : min(b, A.ntiles);
    const uint64_t j0 = min((uint64_t)threadIdx.x * per, jn), j1 = min(j0 + per, jn);
    CFn fb = cf_id(), fa = cf_id();
    for (uint64_t j = j0; j < j1; ++j) {
        const CFn g = A.agg[j];
        if (j < b) fb = cf_compose(fb, g);
        fa = cf_compose(fa, g);
    }
    if constexpr (AM == APPLY_WRAP) {
        if (threadIdx.x == 0) {  // thread 0's aggregates start at tile 0
            CFn low = cf_id();
            const uint64_t nl = A.qv < A.M ? A.qv : A.M;
            for (uint64_t m = 0; m < nl; ++m) low = cf_compose(low, cf_limb(digit(m), A.B));
            if (b > 0) fb = cf_compose(low, fb);
            fa = cf_compose(low, fa);
        }
    }
    CFn ex, before;
    block_scan<SCAN_THREADS>(fb, ex, before);
    uint32_t sel = 0;
    if (A.has_top) {
        CFn all;
        block_scan<SCAN_THREADS>(fa, ex, all);
        const uint64_t tt = digit(A.M);
        const uint32_t ct0 = cf_eval(all, 0u), ct1 = cf_eval(all, 1u);
        sel = (A.dual && ((tt + ct1) >> A.s_top) != 0u) ? 1u : 0u;
        if (b == 0 && threadIdx.x == 0)
            A.out[A.M] = (uint32_t)((tt + (sel ? ct1 : ct0)) & ((1ull << A.s_top) - 1));
    }
    if (b < A.ntiles) {
        CFn f = cf_id();
#pragma unroll
        for (int v = 0; v < CARRY_PER_THREAD; ++v)
            if (base + v < A.M) f = cf_compose(f, cf_limb(tv[v], A.B));
        CFn excl, total;
        block_scan<SCAN_THREADS>(f, excl, total);
        uint32_t carry = cf_eval(excl, cf_eval(before, sel));
        CFn fw = cf_id();
        // FOLD: this thread's limbs in [nlo, Mw] all ones (limb Mw: its s_top bits)
        [[maybe_unused]] const uint64_t nlo = A.Mw < WRAP_LO ? A.Mw : WRAP_LO;
        [[maybe_unused]] const uint32_t topmask = (uint32_t)((1ull << A.s_top) - 1);
        [[maybe_unused]] bool upper_ones = true;
#pragma unroll
        for (int v = 0; v < CARRY_PER_THREAD; ++v) {
            const uint64_t idx = base + v;
            if (idx < A.M) {
                const uint64_t val = tv[v] + carry;
                const uint32_t limb = (uint32_t)(val & mask);
                A.out[idx] = limb;
                carry = (uint32_t)(val >> A.B);
                if constexpr (AM == APPLY_FOLD) {
                    if (idx >= A.qv && idx < A.Mw) fw = cf_compose(fw, cf_limb(limb, A.B));
                    if (idx >= WRAP_LO && idx < A.Mw) A.y[idx] = limb;
                    if (idx == A.Mw) A.y[idx] = limb & topmask;
                    if (idx >= nlo && idx < A.Mw) upper_ones &= limb == (uint32_t)mask;
                    if (idx == A.Mw) upper_ones &= (limb & topmask) == topmask;
                }
                if constexpr (EXTRACT) lb[idx - b * CARRY_TILE] = limb;
                if (EXTRACT && idx + 1 == tile_end) cout = carry;
            }
        }
        if constexpr (AM == APPLY_FOLD) {
            const CFn tw = block_reduce<SCAN_THREADS>(fw);
            if (threadIdx.x == 0) A.agg_w[b] = tw;
            const int ones = __syncthreads_and(upper_ones);
            if (threadIdx.x == 0) A.tflags[b] = ones ? 1u : 0u;
        }
    }
    if constexpr (EXTRACT) {
        if (!A.zout) return;
        const uint32_t st = A.status[1];
        if (b == 0 && threadIdx.x == 0) *A.dst = st;
        if (st != 0u) return;
        __syncthreads();
        if (threadIdx.x == 0) {  // the limbs past the tile, from its carry out
            const uint64_t e0 = b < A.ntiles ? tile_end : 0;
            uint32_t c = b < A.ntiles ? cout : 0u;
            for (uint32_t i = 0; i < EXTRA_LIMBS; ++i) {
                const uint64_t m = e0 + i;
                uint32_t limb = 0;
                if (m < A.M) {
                    const uint64_t v = tx[i] + c;
                    limb = (uint32_t)(v & mask);
                    c = (uint32_t)(v >> A.B);
                } else if (A.has_top && m == A.M) {
                    limb = (uint32_t)((tx[i] + c) & ((1ull << A.s_top) - 1));
                }
                lb[tile_len + i] = limb;
            }
        }
        __syncthreads();
        // output words starting in bits [lo, hi) of the result
        const uint64_t off = A.gamma - A.r;  // bit 0 of z
        const bool last = b + 1 >= max(A.ntiles, (uint64_t)1);
        const uint64_t lo = b * CARRY_TILE * A.B, hi = last ? A.gamma : tile_end * A.B;
        const uint64_t w0 = lo <= off ? 0 : (lo - off + 63) / 64;
        const uint64_t w1 = min(hi <= off ? 0 : (hi - off + 63) / 64, A.out_words);
        for (uint64_t w = w0 + threadIdx.x; w < w1; w += SCAN_THREADS) {
            const uint32_t pos = (uint32_t)(off + 64 * w - lo);  // bit position in lb
            uint64_t v = 0;
            if (A.B == 32) {  // two funnel shifts of three limbs
                const uint32_t j = pos >> 5, sh = pos & 31u;
                const uint32_t l0 = lb[j], l1 = lb[j + 1], l2 = lb[j + 2];
                v = (uint64_t)__builtin_amdgcn_alignbit(l1, l0, sh) |
                    (uint64_t)__builtin_amdgcn_alignbit(l2, l1, sh) << 32;
            } else {
                uint32_t got = 0;
                while (got < 64) {
                    const uint32_t q = pos + got;
                    const uint32_t j = q / A.B;
                    const uint32_t sh = q - j * A.B;
                    const uint32_t take = min(A.B - sh, 64u - got);
                    v |= (((uint64_t)lb[j] >> sh) & ((1ull << take) - 1)) << got;
                    got += take;
                }
            }
            const uint64_t left = A.r - 64 * w;
            if (left < 64) v &= (1ull << left) - 1;
            A.zout[w] = v;
        }
    }
}

template <int AM>
__global__ __launch_bounds__(SCAN_THREADS) void k_carry_apply(ScanArgs A) { carry_apply_body<AM>(A, wg_self()); }

template <int AM>
__global__ __launch_bounds__(SCAN_THREADS) void km_carry_apply(const ScanArgs *__restrict__ tab, const MultiGeo *__restrict__ geo,
                                     const uint16_t *__restrict__ owner) {
    WG wg;
    const uint32_t i = wg_multi(geo, owner, wg);
    if (i != MULTI_NONE) carry_apply_body<AM>(tab[i], wg);
}

// ------------------------------------------------------------------ output

__global__ void k_pack(const uint32_t *__restrict__ limbs, uint64_t *out, uint64_t words, uint64_t gamma,
                       uint32_t B, const uint32_t *status) {
    uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= words || status[1] != 0u) return;
    out[w] = limbs_get64(limbs, B, gamma, 64 * w);
}


inline unsigned blocks_for(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// Launch a kernel of the hash sequence on `st`, or record it (with its
// multi-block form) when the plan records its launches.
template <class Args>
void emit(pa_plan *p, int step, const void *single, const void *multi, dim3 grid, dim3 block, size_t lds,
          const Args &A, hipStream_t st) {
    static_assert(sizeof(Args) <= KARGS_MAX, "argument struct too large to record");
    if (p->rec) {
        p->rec->emplace_back();
        KLaunch &L = p->rec->back();
        L.step = step;
        L.single = single;
        L.multi = multi;
        L.grid = grid;
        L.block = block;
        L.lds = (uint32_t)lds;
        L.args_size = (uint32_t)sizeof(Args);
        std::memcpy(L.args, &A, sizeof(Args));
        return;
    }
    void *args[] = {(void *)&A};
    (void)hipLaunchKernel(single, grid, block, args, lds, st);
}

// The single- and multi-block forms of a kernel instance.
#define PA_KERN(name, ...) (const void *)&k_##name<__VA_ARGS__>, (const void *)&km_##name<__VA_ARGS__>
#define PA_KERN0(name) (const void *)&k_##name, (const void *)&km_##name

// Pair groups of the generic row kernel: rows shorter than 2048 words run
// several pairs side by side, a group per pair with one thread per radix-8
// task (N2/8), up to 256 threads; otherwise one group of N2/16 threads
// (ROW_EPT elements each), at least 64.
unsigned row_groups(const pa_plan *p, uint64_t npairs) {
    const unsigned t = (1u << p->m2) / 8;
    unsigned g = t == 0 || t >= 256 ? 1u : 256u / t;
    return npairs < g ? (unsigned)npairs : g;
}

unsigned row_group_threads(const pa_plan *p, uint64_t npairs) {
    const unsigned n2 = 1u << p->m2;
    if (row_groups(p, npairs) > 1) return n2 / 8;
    const unsigned t = n2 / ROW_EPT;
    return t < 64 ? 64 : t;  // N2 <= 2^14 -> at most 1024 threads
}

// ---------------------------------------------------------------- host math

uint32_t hmul(uint32_t a, uint32_t b, uint32_t p) { return (uint32_t)(((uint64_t)a * b) % p); }

uint32_t hpow(uint32_t b, uint64_t e, uint32_t p) {
    uint32_t r = 1;
    while (e) {
        if (e & 1) r = hmul(r, b, p);
        b = hmul(b, b, p);
        e >>= 1;
    }
    return r;
}

uint32_t hinv(uint32_t a, uint32_t p) { return hpow(a % p, p - 2, p); }

uint32_t hmont(uint32_t a, uint32_t p) { return (uint32_t)(((uint64_t)(a % p) << 32) % p); }

// A primitive 2^log2n-th root of unity (2^log2n | p - 1): g^((p-1)/2^log2n)
// for a quadratic non-residue g, whose order has the full power of two of
// p - 1 (Euler's criterion: g^((p-1)/2) = -1).
uint32_t root_of_unity(uint32_t p, uint32_t log2n) {
    uint32_t g = 2;
    while (hpow(g, (p - 1) / 2, p) != p - 1) ++g;
    return hpow(g, (uint64_t)(p - 1) >> log2n, p);
}

// A primitive root of unity of order f * 2^log2n, f = 1, 3 or 5 (mix 0, 1,
// 2; f * 2^log2n | p - 1).  For f > 1 it is w^a c with w = root_of_unity(p,
// log2n), a = f^-1 mod 2^log2n and c = h^((p-1)/f) != 1 for the smallest such
// h: its f-th power is w itself, so the f power-of-two transforms of the
// radix-f split use exactly the roots (and the radix-16 constants) of the
// plain length-2^log2n transform.
uint32_t root_of_len(uint32_t p, uint32_t log2n, uint32_t mix) {
    const uint32_t w = root_of_unity(p, log2n);
    if (!mix) return w;
    const uint64_t f = len_factor_of(mix);
    uint64_t inv = f;  // f^-1 mod 2^64 by Newton iteration (f * f = 1 mod 8 for f = 3, 5)
    for (int i = 0; i < 5; ++i) inv *= 2 - f * inv;
    const uint64_t a = inv & ((1ull << log2n) - 1);
    uint32_t c = 1;
    for (uint32_t h = 2; c == 1; ++h) c = hpow(h, (p - 1) / (uint32_t)f, p);
    return hmul(hpow(w, a, p), c, p);
}

// The constants of one prime triple at one transform length, computed from
// scratch (modular exponentiations; a few microseconds).
void compute_prime_constants(pa_plan *p, const uint32_t primes[NPRIMES]) {
    for (int q = 0; q < NPRIMES; ++q) {
        const uint32_t pr = primes[q];
        PrimeConst &C = p->primes.c[q];
        C.p = pr;
        uint32_t inv = 1;  // p^-1 mod 2^32 by Newton iteration
        for (int i = 0; i < 5; ++i) inv *= 2u - pr * inv;
        C.pinv = 0u - inv;
        C.one = hmont(1, pr);
        C.p2 = 2u * pr;
        const uint32_t w16 = root_of_unity(pr, 4), w16i = hinv(w16, pr);
        uint32_t a = 1, b = 1;
        for (int j = 0; j < 8; ++j) {
            C.w16[j] = hmont(a, pr);
            C.w16i[j] = hmont(b, pr);
            a = hmul(a, w16, pr);
            b = hmul(b, w16i, pr);
        }
    }
    const uint32_t p0 = primes[0], p1 = primes[1], p2 = primes[2];
    p->crt.inv_p0_mod_p1 = hmont(hinv(p0 % p1, p1), p1);
    p->crt.one_sub = (p0 < 2ull * p1 && p0 < 2ull * p2 && p1 < 2ull * p2) ? 1u : 0u;
    p->crt.inv_p0p1_mod_p2 = hmont(hinv(hmul(p0 % p2, p1 % p2, p2), p2), p2);
    p->crt.inv_p1_mod_p2 = hmont(hinv(p1 % p2, p2), p2);
    p->crt.p0p1 = (uint64_t)p0 * p1;
    for (int q = 0; q < NPRIMES; ++q) {
        const uint32_t pr = primes[q];
        p->mix3.neg_half[q] = hmont((pr - 1) / 2, pr);
        p->mix3.h[q] = 0;
        for (int e = 0; e < 5; ++e) p->mix5.wi[q][e] = 0;
        if (p->mix == 2) {
            const uint32_t w5 = hpow(root_of_len(pr, p->m, 2), p->Nsub, pr);  // omega_N^(N/5) = omega_5
            const uint32_t w5i = hinv(w5, pr);
            uint32_t x = 1;
            for (int e = 0; e < 5; ++e) {
                p->mix5.wi[q][e] = hmont(x, pr);
                x = hmul(x, w5i, pr);
            }
        } else if (p->mix) {
            const uint32_t w3 = hpow(root_of_len(pr, p->m, 1), p->Nsub, pr);  // omega_N^(N/3) = omega_3
            const uint32_t w3sq = hmul(w3, w3, pr);                         // omega_3^-1
            // (omega_3^-1 - omega_3^-2) / 2
            p->mix3.h[q] = hmont(hmul((w3sq + pr - w3) % pr, (pr + 1) / 2, pr), pr);
        }
    }
}

// Prime constants already computed, by (primes, m, mix): a batched call
// derives a plan per block, so each distinct shape pays the exponentiations
// once per process.
struct ConstEntry {
    uint32_t p[NPRIMES], m, mix;
    PrimeSet primes;
    CrtConst crt;
    Mix3Const mix3;
    Mix5Const mix5;
};

}  // namespace

namespace pa {

void init_prime_constants(pa_plan *p, const uint32_t primes[NPRIMES]) {
    static std::mutex mu;
    static std::vector<ConstEntry> cache;
    constexpr size_t kMaxEntries = 256;
    {
        std::lock_guard<std::mutex> lock(mu);
        for (const ConstEntry &e : cache)
            if (e.m == p->m && e.mix == p->mix && e.p[0] == primes[0] && e.p[1] == primes[1] && e.p[2] == primes[2]) {
                p->primes = e.primes;
                p->crt = e.crt;
                p->mix3 = e.mix3;
                p->mix5 = e.mix5;
                return;
            }
    }
    compute_prime_constants(p, primes);
    ConstEntry e{{primes[0], primes[1], primes[2]}, p->m, p->mix, p->primes, p->crt, p->mix3, p->mix5};
    std::lock_guard<std::mutex> lock(mu);
    if (cache.size() < kMaxEntries) cache.push_back(e);
}

hipError_t launch_twiddles(pa_plan *p, hipStream_t st, uint32_t *hdr, uint32_t want) {
    const uint64_t N = p->N, n1 = 1ull << p->m1, n2 = 1ull << p->m2;
    const uint32_t sub = p->rf;  // omega_{N/sub} = omega_N^sub
    TwArgs t1f, t1i, t2f, t2i, Ff, Fi, Gi;
    for (int q = 0; q < NPRIMES; ++q) {
        const uint32_t pr = p->primes.c[q].p;
        const uint32_t w = root_of_len(pr, p->m, p->mix), wi = hinv(w, pr);
        const uint32_t R = (uint32_t)((1ull << 32) % pr);
        t1f.p[q] = t1i.p[q] = t2f.p[q] = t2i.p[q] = Ff.p[q] = Fi.p[q] = Gi.p[q] = pr;
        t1f.base[q] = hpow(w, (uint64_t)sub * n2, pr);  // omega_{N1}
        t1i.base[q] = hpow(wi, (uint64_t)sub * n2, pr);
        t2f.base[q] = hpow(w, (uint64_t)sub * n1, pr);  // omega_{N2}
        t2i.base[q] = hpow(wi, (uint64_t)sub * n1, pr);
        Ff.base[q] = w;
        Fi.base[q] = Gi.base[q] = wi;
        t1f.scale[q] = t1i.scale[q] = t2f.scale[q] = t2i.scale[q] = Ff.scale[q] = Gi.scale[q] = R;
        // inverse four-step twiddle: 1/N, times 2^32 to undo the Montgomery
        // factor of the pointwise product, in Montgomery form
        Fi.scale[q] = hmul(hmul(hinv((uint32_t)(N % pr), pr), R, pr), R, pr);
    }
    hipLaunchKernelGGL(k_tw_pow, dim3(blocks_for(n1, 256), NPRIMES), dim3(256), 0, st, p->tw1f, n1, t1f, hdr, want);
    hipLaunchKernelGGL(k_tw_pow, dim3(blocks_for(n1, 256), NPRIMES), dim3(256), 0, st, p->tw1i, n1, t1i, hdr, want);
    hipLaunchKernelGGL(k_tw_pow, dim3(blocks_for(n2, 256), NPRIMES), dim3(256), 0, st, p->tw2f, n2, t2f, hdr, want);
    hipLaunchKernelGGL(k_tw_pow, dim3(blocks_for(n2, 256), NPRIMES), dim3(256), 0, st, p->tw2i, n2, t2i, hdr, want);
    hipLaunchKernelGGL(k_tw_four, dim3(blocks_for(N / TW4_RUN, 256), NPRIMES), dim3(256), 0, st, p->Wf, p->Wi,
                       p->m1, p->m2, sub, Ff, Fi, hdr, want);
    if (p->mix)
        hipLaunchKernelGGL(k_tw_gx, dim3(blocks_for(p->rf * n1, 256), NPRIMES), dim3(256), 0, st, p->G3, p->rf, p->m1,
                           p->m2, Ff, Gi, hdr, want);
    if (p->m2 == 12) {
        hipLaunchKernelGGL(k_tw_r16, dim3(blocks_for(R16_TW, 256), NPRIMES), dim3(256), 0, st, p->tw2f, p->R16f,
                           hdr, want);
        hipLaunchKernelGGL(k_tw_r16, dim3(blocks_for(R16_TW, 256), NPRIMES), dim3(256), 0, st, p->tw2i, p->R16i,
                           hdr, want);
    }
    if (hdr) hipLaunchKernelGGL(k_tw_mark, dim3(1), dim3(64), 0, st, hdr, want);
    return hipGetLastError();
}

static ColFwdArgs col_args(pa_plan *p, uint32_t mode) {
    ColFwdArgs cf;
    cf.X = p->X;
    cf.N = p->N;
    cf.L = p->L;
    cf.n = p->n;
    cf.gamma = p->gamma;
    cf.k = p->k;
    cf.W = p->W;
    cf.m1 = p->m1;
    cf.m2 = p->m2;
    cf.c_lg = mode == 0 ? p->c_lg : p->c_lg_mh;
    cf.B = p->B;
    cf.s_top = p->s_top;
    cf.mode = mode;
    cf.arr0 = 0;
    cf.key = nullptr;
    cf.a = nullptr;
    cf.b = nullptr;
    cf.ylimbs = nullptr;
    cf.notones = p->notones;
    cf.tw = p->tw1f;
    cf.Nsub = p->Nsub;
    cf.g3 = p->G3;
    cf.P = p->primes;
    return cf;
}

// Column pass of any shape: one workgroup per (tile, array), first-step tasks
// per thread as the tile needs (2^(m1 - 3 + c_lg) tasks, m1 + c_lg <= 14).
// RADIX: the length factor (1, 3 or 5; lengths 5 * 2^m have columns of at
// most 256 rows).
template <int Stage, int RADIX>
static void launch_col_fwd_generic(pa_plan *p, const ColFwdArgs &cf, unsigned narrays, unsigned zsplit,
                                   hipStream_t st) {
    const int step = Stage == STAGE_MMH ? SP_MMH_COL : SP_MH_COL;
    const dim3 grid(1u << (p->m2 - cf.c_lg), narrays, zsplit);
    const size_t col_lds = ((size_t)4 << p->m1) << cf.c_lg;
    const uint32_t ntask = (1u << (p->m1 - 3)) << cf.c_lg;
    // common tile shapes (2^m1 rows x 2^c_lg columns) with compile-time sizes
#define PA_COL_FIXED(LGv, CLGv)                                                                              \
    if constexpr (RADIX != 5 || LGv <= 8) {                                                                  \
        if (p->m1 == LGv && cf.c_lg == CLGv) {                                                               \
            constexpr int NT = 1 << (LGv - (ColR16<LGv, CLGv>::first ? 4 : 3) + CLGv); /* first-step tasks */\
            constexpr int T = NT <= COL_THREADS ? 1 : NT / COL_THREADS;                                      \
            emit(p, step, PA_KERN(col_fwd, Stage, RADIX, T, LGv, CLGv), grid, dim3(COL_THREADS), 0, cf, st);\
            return;                                                                                          \
        }                                                                                                    \
    }
    PA_COL_FIXED(3, 4) PA_COL_FIXED(3, 7) PA_COL_FIXED(3, 8)
    PA_COL_FIXED(4, 4) PA_COL_FIXED(4, 6) PA_COL_FIXED(4, 7)
    PA_COL_FIXED(5, 4) PA_COL_FIXED(5, 6)
    PA_COL_FIXED(6, 4) PA_COL_FIXED(6, 5)
    PA_COL_FIXED(7, 4) PA_COL_FIXED(8, 4) PA_COL_FIXED(10, 3) PA_COL_FIXED(10, 4)
#undef PA_COL_FIXED
    if (ntask <= COL_THREADS)
        emit(p, step, PA_KERN(col_fwd, Stage, RADIX, 1), grid, dim3(COL_THREADS), col_lds, cf, st);
    else if (ntask <= 2 * COL_THREADS)
        emit(p, step, PA_KERN(col_fwd, Stage, RADIX, 2), grid, dim3(COL_THREADS), col_lds, cf, st);
    else if (ntask <= 4 * COL_THREADS)
        emit(p, step, PA_KERN(col_fwd, Stage, RADIX, 4), grid, dim3(COL_THREADS), col_lds, cf, st);
    else
        emit(p, step, PA_KERN(col_fwd, Stage, RADIX, 8), grid, dim3(COL_THREADS), col_lds, cf, st);
}

// zsplit (1 or 3) workgroups share a tile's transforms, each taking the
// primes (and radix-3 or radix-5 branches) of its slice: more workgroups for
// passes with few arrays, at the cost of unpacking the tile's limbs once per
// slice.
template <int Stage>
static void launch_col_fwd(pa_plan *p, const ColFwdArgs &cf, unsigned narrays, unsigned zsplit, hipStream_t st) {
    const unsigned ncol_tiles = 1u << (p->m2 - cf.c_lg);
    const bool c9 = p->m1 == C9_LG && cf.c_lg == C9_CLG;  // 512 x 16 tiles in static LDS
    // 1024 x 8 tiles in static LDS: for 2^m lengths and the MH stage (measured
    // faster there); the radix-3 key-chunk pass runs the generic kernel's
    // compile-time 1024 x 8 instance, which measured faster for it
    const bool c10 = p->m1 == C10_LG && cf.c_lg == C10_CLG && (!p->mix || Stage == STAGE_MH);
    const int step = Stage == STAGE_MMH ? SP_MMH_COL : SP_MH_COL;
    const dim3 grid(ncol_tiles, narrays, zsplit);
    if (p->rf == 5)  // columns of at most 256 rows
        launch_col_fwd_generic<Stage, 5>(p, cf, narrays, zsplit, st);
    else if (c10 && p->mix)
        emit(p, step, PA_KERN(col10_fwd, Stage, true), grid, dim3(COL_THREADS), 0, cf, st);
    else if (c10)
        emit(p, step, PA_KERN(col10_fwd, Stage, false), grid, dim3(COL_THREADS), 0, cf, st);
    else if (c9 && p->mix)  // three primes and radix-3 transforms per tile
        emit(p, step, PA_KERN(col9_fwd, Stage, true), grid, dim3(c9f_threads(Stage, true)), 0, cf, st);
    else if (c9)  // three primes per tile
        emit(p, step, PA_KERN(col9_fwd, Stage, false), grid, dim3(c9f_threads(Stage, false)), 0, cf, st);
    else if (p->mix)
        launch_col_fwd_generic<Stage, 3>(p, cf, narrays, zsplit, st);
    else
        launch_col_fwd_generic<Stage, 1>(p, cf, narrays, zsplit, st);
}

static RowArgs row_args(pa_plan *p, uint64_t npairs, const uint32_t *seed_side) {
    RowArgs ra;
    ra.X = p->X;
    ra.A = seed_side;
    ra.N = p->N;
    ra.npairs = npairs;
    ra.pair_stride = (uint64_t)NPRIMES * p->N;
    ra.m2 = p->m2;
    ra.out = p->Cc;
    ra.Wf = p->Wf;
    ra.Wi = p->Wi;
    ra.twf = p->tw2f;
    ra.twi = p->tw2i;
    ra.r16f = p->R16f;
    ra.r16i = p->R16i;
    ra.row_group = row_group_threads(p, npairs);
    ra.P = p->primes;
    return ra;
}

template <int Stage>
static void launch_row(pa_plan *p, const RowArgs &ra, hipStream_t st) {
    const unsigned rows = (unsigned)(p->N >> p->m2);  // 2^m1, or 3 * 2^m1 for N = 3 * 2^m
    const int step = Stage == STAGE_MMH ? SP_MMH_ROW : SP_MH_ROW;
    if (p->m2 == 12) {
        emit(p, step, PA_KERN(row16, Stage), dim3(rows, NPRIMES), dim3(R16_THREADS), 0, ra, st);
    } else {
        const unsigned groups = row_groups(p, ra.npairs);
        // groups of at most a wavefront synchronise their steps within it
        if (ra.row_group <= 64)
            emit(p, step, PA_KERN(row, Stage, true), dim3(rows, NPRIMES), dim3(groups * ra.row_group),
                 (size_t)groups * 4 << p->m2, ra, st);
        else
            emit(p, step, PA_KERN(row, Stage, false), dim3(rows, NPRIMES), dim3(groups * ra.row_group),
                 (size_t)groups * 4 << p->m2, ra, st);
    }
}

static ColInvArgs colinv_args(pa_plan *p) {
    ColInvArgs ci;
    ci.Cc = p->Cc;
    ci.N = p->N;
    ci.m1 = p->m1;
    ci.m2 = p->m2;
    ci.c_lg = p->ci_lg;
    ci.twi = p->tw1i;
    ci.Nsub = p->Nsub;
    ci.row_lim = 1u << p->m1;
    ci.P = p->primes;
    return ci;
}

template <int Stage>
static void launch_col_inv(pa_plan *p, const ColInvArgs &ci, hipStream_t st) {
    const unsigned nsub = p->rf;  // grid z: transform of the radix-3 or radix-5 split
    const int step = Stage == STAGE_MMH ? SP_MMH_COLINV : SP_MH_COLINV;
    if (p->m1 == C9_LG && p->m2 >= C9_CLG)
        emit(p, step, PA_KERN(col9_inv, Stage), dim3(1u << (p->m2 - C9_CLG), NPRIMES, nsub), dim3(C9I_THREADS), 0,
             ci, st);
    else if (p->m1 == C10_LG && p->m2 >= C10_CLG)
        emit(p, step, PA_KERN(col10_inv, Stage), dim3(1u << (p->m2 - C10_CLG), NPRIMES, nsub), dim3(COL_THREADS),
             0, ci, st);
    else if (p->m1 == 7 && p->m2 >= 5)  // 128 x 32 tiles, two LDS passes
        emit(p, step, PA_KERN(col_inv16, Stage, 7, 5), dim3(1u << (p->m2 - 5), NPRIMES, nsub), dim3(COL_THREADS), 0,
             ci, st);
    else if (p->m1 == 8 && p->m2 >= 4)  // 256 x 16 tiles, two LDS passes
        emit(p, step, PA_KERN(col_inv16, Stage, 8, 4), dim3(1u << (p->m2 - 4), NPRIMES, nsub), dim3(COL_THREADS), 0,
             ci, st);
    else
        emit(p, step, PA_KERN(col_inv, Stage), dim3(1u << (p->m2 - p->ci_lg), NPRIMES, nsub), dim3(COL_THREADS),
             ((size_t)4 << p->m1) << p->ci_lg, ci, st);
}

hipError_t launch_mmh(pa_plan *p, const uint64_t *key, const uint64_t *a, hipStream_t st) {
    ColFwdArgs cf = col_args(p, 0);
    cf.key = key;
    cf.a = a;
    phase_mark(p, PA_PH_MMH_COL, true, st);
    // with resident seed transforms only the k key chunks are transformed
    launch_col_fwd<STAGE_MMH>(p, cf, (unsigned)(p->res_a ? p->k : 2 * p->k), 1u, st);
    phase_mark(p, PA_PH_MMH_COL, false, st);

    RowArgs ra = row_args(p, p->k, p->res_a ? p->res_a : p->X + p->k * NPRIMES * p->N);
    phase_mark(p, PA_PH_MMH_ROW, true, st);
    launch_row<STAGE_MMH>(p, ra, st);
    phase_mark(p, PA_PH_MMH_ROW, false, st);

    ColInvArgs ci = colinv_args(p);
    phase_mark(p, PA_PH_MMH_COLINV, true, st);
    launch_col_inv<STAGE_MMH>(p, ci, st);
    phase_mark(p, PA_PH_MMH_COLINV, false, st);
    return hipGetLastError();
}

static DigitArgs digit_args(pa_plan *p) {
    DigitArgs A;
    A.c96 = p->C96;
    A.cseed = nullptr;
    A.fix = WrapFix{};
    A.t = p->t;
    A.agg = p->agg;
    A.N = p->N;
    A.L = p->L;
    A.ncoef = 2 * p->L - 1;  // nonzero coefficients of the product
    A.gamma = p->gamma;
    A.B = p->B;
    A.e = p->e_fold;
    A.Q = (96 + p->B - 1) / p->B;
    A.Q2 = (96 + p->e_fold + p->B - 1) / p->B;
    A.s_top = p->s_top;
    return A;
}

static ScanArgs scan_args(pa_plan *p, uint32_t *out, uint64_t M, bool top, bool dual) {
    ScanArgs S{};
    S.t = p->t;
    S.out = out;
    S.M = M;
    S.B = p->B;
    S.has_top = top ? 1u : 0u;
    S.s_top = p->s_top;
    S.dual = dual ? 1u : 0u;
    S.ntiles = (M + CARRY_TILE - 1) / CARRY_TILE;
    S.agg = p->agg;
    S.agg_w = p->agg_w;
    S.Mw = p->L - 1;
    S.s = p->s;
    S.gamma = p->gamma;
    S.M1 = p->M1;
    S.qv = (128 + p->B - 1) / p->B;
    S.y = p->y;
    S.flag = p->status + 2;  // the second fold's general case is needed
    S.wrapinfo = p->status + 3;
    S.tflags = p->tflags;
    return S;
}

// The first fold's extra workgroup writes y's lowest limbs itself when
// V mod p fits below limb min(32, L - 1) (ceil(128 / B) limbs), always true
// but for the smallest blocks.
bool wrap_inline(const pa_plan *p) {
    const uint64_t nlo = std::min<uint64_t>(WRAP_LO, p->L - 1);
    return (128 + p->B - 1) / p->B < nlo;
}

// FOLD: one workgroup more than the tiles (the second fold's usual case).
// WRAP: at most WRAP_GRID workgroups, looping over the tiles.
constexpr uint64_t WRAP_GRID = 128;

template <int AM>
static void launch_apply(pa_plan *p, const ScanArgs &S, hipStream_t st) {
    const uint64_t nt = S.ntiles ? S.ntiles : 1;
    const uint64_t wg = AM == APPLY_FOLD ? S.ntiles + 1 : AM == APPLY_WRAP ? std::min(nt, WRAP_GRID) : nt;
    const int step = AM == APPLY_FOLD ? SP_FOLD_APPLY : AM == APPLY_WRAP ? SP_FOLD_WRAP : SP_MH_APPLY;
    emit(p, step, PA_KERN(carry_apply, AM), dim3((unsigned)wg), dim3(SCAN_THREADS), 0, S, st);
}

// Carry normalisation of the digit sums A.t[0..M) (plus the top limb at M if
// top) into `out`: the tile kernel (digits and tile aggregates), then apply
// (for FOLD also the wrap chain's tile aggregates).  With `crt` the digits
// come straight from the residues (k_digit_crt, for N = 2^m), else from the
// coefficient word planes.
template <int MODE>
static hipError_t run_carry(pa_plan *p, DigitArgs A, uint32_t *out, uint64_t ndig, uint64_t M, bool top,
                            bool dual, hipStream_t st, DigitCrtArgs *crt, uint64_t *zout = nullptr,
                            uint32_t *dst = nullptr) {
    A.ndig = ndig;
    A.M = M;
    const uint64_t tiles_t = (ndig + CARRY_TILE - 1) / CARRY_TILE;
    const int step = MODE == DIG_FOLD ? SP_FOLD_DIGIT : SP_MH_DIGIT;
    if (tiles_t && crt) {
        crt->D = A;
        emit(p, step, PA_KERN(digit_crt, MODE), dim3((unsigned)tiles_t), dim3(DIG_THREADS), 0, *crt, st);
    } else if (tiles_t) {
        emit(p, step, PA_KERN(digit_tile, MODE), dim3((unsigned)tiles_t), dim3(DIG_THREADS), 0, A, st);
    }
    ScanArgs S = scan_args(p, out, M, top, dual);
    S.zout = zout;  // MH: the output extraction rides on the apply
    S.out_words = p->out_words;
    S.r = p->r;
    S.status = p->status;
    S.dst = dst;
    launch_apply<MODE == DIG_FOLD ? APPLY_FOLD : APPLY_PLAIN>(p, S, st);
    return hipGetLastError();
}

// The hash status check for the fold's reconstruction kernel; seeds nullptr
// (the MH stage): none.
static StatusArgs status_args(pa_plan *p, const Seeds *seeds) {
    StatusArgs S{};
    if (!seeds) return S;
    S.a = seeds->a;
    S.b = seeds->b;
    S.c = seeds->c;
    S.k = p->k;
    S.W = p->W;
    S.gamma = p->gamma;
    S.notones = p->notones;
    S.nt = 1u << (p->m2 - p->c_lg);  // column tiles of the key-chunk pass
    S.status = p->status;
    return S;
}

// Coefficients [0, count) of the convolution for N = 3 * 2^m from the
// residues in Cc, as word planes in C96 (with notones: also the RELOAD
// status).  For N = 2^m the digit kernels reconstruct the coefficients.
static void launch_crt5(pa_plan *p, uint64_t count, const Seeds *seeds, int step, hipStream_t st) {
    Crt5Args A;
    A.cc = p->Cc;
    A.c96 = p->C96;
    A.N = p->N;
    A.Nsub = p->Nsub;
    A.count = count;
    A.m1 = p->m1;
    A.m2 = p->m2;
    A.gi = p->G3 + (size_t)3 * NPRIMES * 5 * ((size_t)1 << p->m1);  // after the three forward tables
    A.P = p->primes;
    A.K = p->crt;
    A.X = p->mix5;
    A.S = status_args(p, seeds);
    emit(p, step, PA_KERN0(crt5), dim3(blocks_for(count < p->Nsub ? count : p->Nsub, 256)), dim3(256), 0, A, st);
}

static void launch_crt3(pa_plan *p, uint64_t count, const Seeds *seeds, int step, hipStream_t st) {
    if (p->rf == 5) {
        launch_crt5(p, count, seeds, step, st);
        return;
    }
    Crt3Args A;
    A.cc = p->Cc;
    A.c96 = p->C96;
    A.N = p->N;
    A.Nsub = p->Nsub;
    A.count = count;
    A.m1 = p->m1;
    A.m2 = p->m2;
    A.gi = p->G3 + (size_t)2 * NPRIMES * 3 * ((size_t)1 << p->m1);
    A.P = p->primes;
    A.K = p->crt;
    A.X = p->mix3;
    A.S = status_args(p, seeds);
    emit(p, step, PA_KERN0(crt3), dim3(blocks_for(count < p->Nsub ? count : p->Nsub, 256)), dim3(256), 0, A, st);
}

// Reconstruction inside the digit kernel (N = 2^m); nullptr for N = 3 * 2^m,
// whose coefficients need the inverse radix-3 step of k_crt3 first.
static DigitCrtArgs *residue_digits(pa_plan *p, DigitCrtArgs &C, const Seeds *seeds) {
    if (p->mix) return nullptr;
    C.cc = p->Cc;
    C.P = p->primes;
    C.K = p->crt;
    C.S = status_args(p, seeds);
    return &C;
}

hipError_t launch_fold(pa_plan *p, const Seeds &seeds, hipStream_t st) {
    phase_mark(p, PA_PH_FOLD, true, st);
    const uint64_t ncoef = 2 * p->L - 1;  // nonzero coefficients of the product
    DigitCrtArgs C;
    DigitCrtArgs *crt = residue_digits(p, C, &seeds);
    if (!crt) launch_crt3(p, ncoef, &seeds, SP_FOLD_CRT3, st);
    // first fold at bit gamma, normalised over M1 digits (the sum fits: no carry out);
    // its apply also writes y for the second fold's usual case (V mod p changes only
    // the lowest limbs) and sets a flag when that case does not apply
    hipError_t e = run_carry<DIG_FOLD>(p, digit_args(p), p->s, p->M1, p->M1, false, false, st, crt);
    if (e != hipSuccess) return e;
    // without the inline form (the lowest limbs cannot hold V mod p), the
    // general case runs here (see launch_wrap); with it, the MH digits settle
    // the rare case (WrapFix) and y itself is recomputed only for pa_hash_stages
    if (!wrap_inline(p)) (void)launch_wrap(p, st);
    e = hipGetLastError();
    phase_mark(p, PA_PH_FOLD, false, st);
    return e;
}

hipError_t launch_wrap(pa_plan *p, hipStream_t st) {
    // second fold, general case (runs only when flagged): y = T_lo + (V mod p) over L
    // limbs, straight from the limbs of the first (whose apply left the wrap chain's
    // tile aggregates); the dual evaluation (carry-in 0 or 1) selects S or
    // S + 1 - 2^gamma, which maps a sum equal to p to 0
    ScanArgs S = scan_args(p, p->y, p->L - 1, true, true);
    S.agg = p->agg_w;
    launch_apply<APPLY_WRAP>(p, S, st);
    return hipGetLastError();
}

hipError_t launch_mh(pa_plan *p, const uint64_t *b, const uint64_t *c, uint64_t *out, uint32_t *d_status,
                     hipStream_t st) {
    ColFwdArgs cf = col_args(p, 1);
    cf.b = b;
    cf.ylimbs = p->y;
    phase_mark(p, PA_PH_MH_COL, true, st);
    // one or two arrays: a workgroup per prime fills the GPU
    launch_col_fwd<STAGE_MH>(p, cf, p->res_b ? 1u : 2u, MH_COL_ZSPLIT, st);
    phase_mark(p, PA_PH_MH_COL, false, st);

    RowArgs ra = row_args(p, 1, p->res_b ? p->res_b : p->X + (uint64_t)NPRIMES * p->N);
    phase_mark(p, PA_PH_MH_ROW, true, st);
    launch_row<STAGE_MH>(p, ra, st);
    phase_mark(p, PA_PH_MH_ROW, false, st);

    ColInvArgs ci = colinv_args(p);
    // mod 2^gamma only the coefficients below limb L count: rows below ceil(L / N2)
    // (with N = 3 * 2^m every row of the three transforms feeds some of them)
    if (!p->mix) ci.row_lim = (uint32_t)((p->L + (1ull << p->m2) - 1) >> p->m2);
    phase_mark(p, PA_PH_MH_COLINV, true, st);
    launch_col_inv<STAGE_MH>(p, ci, st);
    phase_mark(p, PA_PH_MH_COLINV, false, st);

    phase_mark(p, PA_PH_MH_CARRY, true, st);
    // only the coefficients below limb L matter mod 2^gamma
    DigitCrtArgs C;
    DigitCrtArgs *crt = residue_digits(p, C, nullptr);
    if (!crt) launch_crt3(p, p->L, nullptr, SP_MH_CRT3, st);
    DigitArgs A = digit_args(p);
    A.cseed = c;
    if (wrap_inline(p)) A.fix = WrapFix{b, p->status + 3, p->tflags, (p->M1 + CARRY_TILE - 1) / CARRY_TILE};
    // the apply also extracts z and copies the status flags out
    hipError_t e = run_carry<DIG_MH>(p, A, p->U, p->L, p->L - 1, true, false, st, crt, out,
                                     d_status ? d_status : p->status_out);
    phase_mark(p, PA_PH_MH_CARRY, false, st);
    return e;
}

hipError_t launch_fill(uint32_t *dst, uint64_t count, uint32_t word, hipStream_t st) {
    if (count == 0) return hipSuccess;
    const uint64_t groups = std::min<uint64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill32, dim3((unsigned)groups), dim3(256), 0, st, dst, count, word);
    return hipGetLastError();
}

hipError_t launch_finish(pa_plan *p, uint64_t *y_out, uint64_t *U_out, hipStream_t st) {
    phase_mark(p, PA_PH_FINISH, true, st);
    if (y_out)
        hipLaunchKernelGGL(k_pack, dim3(blocks_for(p->W, 256)), dim3(256), 0, st, p->y, y_out, p->W, p->gamma,
                           p->B, p->status);
    if (U_out)
        hipLaunchKernelGGL(k_pack, dim3(blocks_for(p->W, 256)), dim3(256), 0, st, p->U, U_out, p->W, p->gamma,
                           p->B, p->status);
    phase_mark(p, PA_PH_FINISH, false, st);
    return hipGetLastError();
}

// Column-pass outputs of a session's seeds, computed once and kept: the k_max
// seed chunks a_i (MMH stage) into dst_a (k_max x 3 x N words) and b (MH
// stage) into dst_b (3 x N words), for transforms of p's shape.  A hash with
// p->res_a / p->res_b set then transforms only its key chunks and y.
hipError_t launch_seed_transforms(pa_plan *p, const uint64_t *a, uint64_t kmax, const uint64_t *b,
                                  uint32_t *dst_a, uint32_t *dst_b, hipStream_t st) {
    ColFwdArgs cf = col_args(p, 0);
    cf.X = dst_a;
    cf.k = kmax;
    cf.arr0 = (uint32_t)kmax;  // arrays kmax .. 2 kmax - 1 are the seed chunks
    cf.a = a;
    launch_col_fwd<STAGE_MMH>(p, cf, (unsigned)kmax, 1u, st);
    ColFwdArgs cb = col_args(p, 1);
    cb.X = dst_b;
    cb.arr0 = 1;  // array 1 of the MH stage is b
    cb.b = b;
    launch_col_fwd<STAGE_MH>(p, cb, 1u, MH_COL_ZSPLIT, st);
    return hipGetLastError();
}

}  // namespace pa
