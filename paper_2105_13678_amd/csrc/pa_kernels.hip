// HIP kernels of the MMH-MH hash for gfx950 (CDNA4, 64-wide wavefronts).
//
// Pipeline for one block (Algorithm 1 of arXiv 2105.13678):
//   MMH (Sec. 2.1 eq. 2): unpack key chunks x_i and seeds a_i into B-bit limbs,
//        forward NTT of all 2k limb arrays, pointwise multiply-accumulate
//        sum_i A_i * X_i in the transform domain, one inverse NTT -> exact
//        coefficients of S = sum_i a_i x_i.
//   fold (Sec. 3.1, x mod M = floor(x/2^gamma) + x mod 2^gamma): fold the
//        coefficients above bit gamma onto the low part, carry-normalise,
//        fold the small overflow back and canonicalise -> y in [0, p).
//   MH (Sec. 2.2 eq. 4): NTT product b*y, add c while carrying the low gamma
//        bits, keep bits [gamma - r, gamma) -> z.
//
// NTT of length N = N1 * N2 (four-step): a column pass does length-N1 DIF
// transforms on strided columns (LDS tile of 2^c_lg columns), a row pass does
// the twiddle multiply and length-N2 DIF transforms on contiguous rows.  The
// MMH row pass transforms x_i and a_i rows, accumulates their product over i
// and immediately runs the inverse row transform on the accumulated row, so
// the transform-domain sum never goes back to HBM.  The inverse column pass
// (DIT) returns natural-order coefficients; 1/N is folded into the inverse
// twiddles.
//
// Carry propagation uses carry transfer functions f(c) = g + [c >= th]
// (exact for carries below 2^B), composed with wavefront shuffles inside a
// workgroup and a reduce / tile-prefix / apply sequence across workgroups.
#include "ntt_device.hpp"
#include "pa_internal.hpp"

using namespace pa;

extern __shared__ uint64_t lds_dyn[];

namespace {

constexpr int COL_THREADS = 256;
constexpr int ROW_EPT = 16;  // row elements per thread
constexpr int PREFIX_THREADS = 1024;

__device__ __forceinline__ uint32_t bitrev(uint32_t x, uint32_t bits) {
    return bits ? (__brev(x) >> (32 - bits)) : 0u;
}

// Workgroup b of a G-workgroup grid is dispatched to XCD b % 8; hand each XCD
// a contiguous range of tiles so neighbouring tiles share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t G) {
    uint32_t x = b & 7u, i = b >> 3;
    uint32_t q = G >> 3, rr = G & 7u;
    return x * q + min(x, rr) + i;
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

// ------------------------------------------------------------------ twiddles

__global__ void k_tw_pow(uint64_t *dst, uint64_t count, uint64_t base) {
    uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count) dst[j] = gl_pow(base, j);
}

// Four-step twiddles in stored row order: row rho holds frequency
// k1 = bitrev(rho); Wf = omega_N^(k1*n2), Wi = N^-1 * omega_N^-(k1*n2).
__global__ void k_tw_four(uint64_t *Wf, uint64_t *Wi, uint32_t m1, uint32_t m2, uint64_t w,
                          uint64_t winv, uint64_t ninv) {
    uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >> (m1 + m2)) return;
    uint32_t rho = (uint32_t)(idx >> m2);
    uint32_t n2 = (uint32_t)(idx & ((1u << m2) - 1));
    uint64_t e = (uint64_t)bitrev(rho, m1) * n2;
    Wf[idx] = gl_pow(w, e);
    Wi[idx] = gl_mul(ninv, gl_pow(winv, e));
}

// ------------------------------------------------------------------ status

// Clears the chunk flags and checks the seeds: any bit >= gamma in a seed
// word -> SEED_RANGE; even b -> B_EVEN (MH needs gcd(b, 2) = 1).
__global__ void k_prologue(const uint64_t *a, const uint64_t *b, const uint64_t *c, uint64_t k,
                           uint64_t W, uint64_t gamma, uint32_t *notones, uint32_t *status) {
    uint64_t topmask = (gamma & 63) ? ((1ull << (gamma & 63)) - 1) : ~0ull;
    bool range = false;
    for (uint64_t i = threadIdx.x; i < k; i += blockDim.x) {
        notones[i] = 0u;
        range |= (a[i * W + W - 1] & ~topmask) != 0;
    }
    if (threadIdx.x == 0) range |= ((b[W - 1] | c[W - 1]) & ~topmask) != 0;
    int any = __syncthreads_or(range);
    if (threadIdx.x == 0) {
        uint32_t f = any ? ST_SEED_RANGE : 0u;
        if ((b[0] & 1ull) == 0) f |= ST_B_EVEN;
        status[0] = f;
        status[1] = 0u;
    }
}

// After the MMH column pass: RELOAD if some chunk had only all-ones limbs.
__global__ void k_status(const uint32_t *notones, uint64_t k, uint32_t *status) {
    bool reload = false;
    for (uint64_t i = threadIdx.x; i < k; i += blockDim.x) reload |= (notones[i] == 0u);
    int any = __syncthreads_or(reload);
    if (threadIdx.x == 0) status[1] = status[0] | (any ? ST_RELOAD : 0u);
}

// ------------------------------------------------------------------ NTT passes

struct ColFwdArgs {
    uint64_t *X;
    uint64_t N, L, n, gamma, k, W;
    uint32_t m1, m2, c_lg, B, s_top, mode;  // mode 0: MMH (key chunks, seed chunks); 1: MH (y, b)
    const uint64_t *key, *a, *b;
    const uint32_t *ylimbs;
    uint32_t *notones;
    const uint64_t *tw;  // omega_{N1}^e, e < N1
};

// Unpack + forward column pass.  blockIdx.y selects the array: in MMH mode
// arrays 0..k-1 are the key chunks x_i and k..2k-1 the seed chunks a_i; in
// MH mode array 0 is y and array 1 is b.  Limb j of a chunk is its bits
// [jB, jB+B); limbs j >= L are the zero padding.  Because N >= 2L - 1, every
// limb index >= N/2 is padding, so rows n1 >= N1/2 of the column tile are
// zero and the first radix-8 step only unpacks its lower four inputs.
__global__ __launch_bounds__(COL_THREADS) void k_col_fwd(ColFwdArgs A) {
    uint64_t *lds = lds_dyn;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t arr = blockIdx.y;
    const uint32_t c_lg = A.c_lg, lg = A.m1;
    const uint32_t cmask = (1u << c_lg) - 1;
    const uint64_t c0 = (uint64_t)tile << c_lg;
    const bool is_key = (A.mode == 0) && arr < A.k;
    const uint32_t full = (1u << A.B) - 1, topv = (1u << A.s_top) - 1;
    const uint32_t lgMp = lg - 3;
    const uint32_t ntask = (1u << lgMp) << c_lg;
    bool not_ones = false;
    for (uint32_t task = threadIdx.x; task < ntask; task += blockDim.x) {
        const uint32_t q = task & cmask;
        const uint32_t n1 = task >> c_lg;
        uint64_t v[8];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const uint64_t row = n1 + ((uint64_t)jj << lgMp);
            const uint64_t j = (row << A.m2) + c0 + q;  // limb index
            uint32_t x = 0;
            if (j < A.L) {
                if (A.mode == 0) {
                    if (arr < A.k) {
                        const uint64_t base = (uint64_t)arr * A.gamma;
                        const uint64_t lim = min(A.n, base + A.gamma);
                        x = bits_at(A.key, lim, base + j * A.B, A.B);
                        not_ones |= (x != (j == A.L - 1 ? topv : full));
                    } else {
                        x = bits_at(A.a + (uint64_t)(arr - A.k) * A.W, A.gamma, j * A.B, A.B);
                    }
                } else {
                    x = (arr == 0) ? A.ylimbs[j] : bits_at(A.b, A.gamma, j * A.B, A.B);
                }
            }
            v[jj] = x;
        }
        dft_fwd8_lowhalf(v);
        if (lg > 3) {
#pragma unroll
            for (int s = 1; s < 8; ++s) v[s] = fmul(v[s], A.tw[n1 * brev_small(s, 3)]);
        }
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) lds[swz(((n1 + ((uint32_t)jj << lgMp)) << c_lg) + q)] = v[jj];
    }
    if (is_key) {
        int any = __syncthreads_or(not_ones);
        if (any && threadIdx.x == 0) A.notones[arr] = 1u;
    } else {
        __syncthreads();
    }
    fwd_steps_from(lds, lg, lg - 3, c_lg, A.tw, threadIdx.x, blockDim.x);
    uint64_t *out = A.X + (uint64_t)arr * A.N;
    const uint32_t cnt = (1u << lg) << c_lg;
    for (uint32_t e = threadIdx.x; e < cnt; e += blockDim.x)
        out[((uint64_t)(e >> c_lg) << A.m2) + c0 + (e & cmask)] = lds[swz(e)];
}

struct RowArgs {
    const uint64_t *X;
    uint64_t N, npairs, a_off;
    uint32_t m2;
    uint64_t *out;
    const uint64_t *Wf, *Wi, *twf, *twi;  // four-step twiddles; omega_{N2}^{+-e}, e < N2
};

// First forward step of a row straight from global memory: four-step
// twiddle on load, radix-8 DFT, step twiddles, into LDS.
__device__ __forceinline__ void row_first_step(const uint64_t *__restrict__ g, const uint64_t *__restrict__ w,
                                               uint64_t *buf, uint32_t lg, const uint64_t *__restrict__ tw,
                                               uint32_t tid, uint32_t nt) {
    const uint32_t lgMp = lg - 3;
    for (uint32_t n1 = tid; n1 < (1u << lgMp); n1 += nt) {
        uint64_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t e = n1 + ((uint32_t)j << lgMp);
            v[j] = fmul(g[e], w[e]);
        }
        dft_fwd<8>(v);
        if (lg > 3) {
#pragma unroll
            for (int s = 1; s < 8; ++s) v[s] = fmul(v[s], tw[n1 * brev_small(s, 3)]);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) buf[swz(n1 + ((uint32_t)j << lgMp))] = v[j];
    }
    __syncthreads();
}

// Last inverse step of a row straight to global memory (with the inverse
// four-step twiddle and 1/N).
__device__ __forceinline__ void row_last_inv_step(const uint64_t *buf, uint64_t *__restrict__ g,
                                                  const uint64_t *__restrict__ w, uint32_t lg,
                                                  const uint64_t *__restrict__ twi, uint32_t tid, uint32_t nt) {
    const uint32_t lgMp = lg - 3;
    for (uint32_t n1 = tid; n1 < (1u << lgMp); n1 += nt) {
        uint64_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = buf[swz(n1 + ((uint32_t)j << lgMp))];
        if (lg > 3) {
#pragma unroll
            for (int s = 1; s < 8; ++s) v[s] = fmul(v[s], twi[n1 * brev_small(s, 3)]);
        }
        dft_inv<8>(v);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t e = n1 + ((uint32_t)j << lgMp);
            g[e] = fmul(v[j], w[e]);
        }
    }
}

// Row pass: for each pair (x_i, a_i): four-step twiddle and forward transform
// of both rows, accumulate their pointwise product; then the inverse
// transform of the accumulated row, inverse twiddle (with 1/N), store.
__global__ __launch_bounds__(512) void k_row(RowArgs A) {
    uint64_t *lds = lds_dyn;
    const uint32_t lg = A.m2;
    const uint32_t N2 = 1u << lg;
    const uint32_t T = blockDim.x;
    const uint32_t rho = xcd_tile(blockIdx.x, gridDim.x);
    const uint64_t rbase = (uint64_t)rho << lg;
    const uint64_t *wf = A.Wf + rbase;
    uint64_t acc[ROW_EPT], xr[ROW_EPT];
#pragma unroll
    for (int q = 0; q < ROW_EPT; ++q) {
        acc[q] = 0ull;
        xr[q] = 0ull;
    }
    for (uint64_t i = 0; i < A.npairs; ++i) {
        const uint64_t *xrow = A.X + i * A.N + rbase;
        const uint64_t *arow = xrow + A.a_off;
        row_first_step(xrow, wf, lds, lg, A.twf, threadIdx.x, T);
        fwd_steps_from(lds, lg, lg - 3, 0, A.twf, threadIdx.x, T);
#pragma unroll
        for (int q = 0; q < ROW_EPT; ++q) {
            uint32_t e = threadIdx.x + q * T;
            if (e < N2) xr[q] = lds[swz(e)];
        }
        __syncthreads();
        row_first_step(arow, wf, lds, lg, A.twf, threadIdx.x, T);
        fwd_steps_from(lds, lg, lg - 3, 0, A.twf, threadIdx.x, T);
#pragma unroll
        for (int q = 0; q < ROW_EPT; ++q) {
            uint32_t e = threadIdx.x + q * T;
            if (e < N2) acc[q] = fadd(acc[q], fmul(xr[q], lds[swz(e)]));
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < ROW_EPT; ++q) {
        uint32_t e = threadIdx.x + q * T;
        if (e < N2) lds[swz(e)] = acc[q];
    }
    __syncthreads();
    inv_steps_to(lds, lg, lg - 3, 0, A.twi, threadIdx.x, T);
    row_last_inv_step(lds, A.out + rbase, A.Wi + rbase, lg, A.twi, threadIdx.x, T);
}

struct ColInvArgs {
    uint64_t *Cc;
    uint32_t m1, m2, c_lg;
    const uint64_t *twi;  // omega_{N1}^-e, e < N1
};

// Inverse column pass (bit-reversed rows in, natural rows out), in place.
__global__ __launch_bounds__(COL_THREADS) void k_col_inv(ColInvArgs A) {
    uint64_t *lds = lds_dyn;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t c_lg = A.c_lg, lg = A.m1;
    const uint32_t cmask = (1u << c_lg) - 1;
    const uint32_t cnt = (1u << lg) << c_lg;
    const uint64_t c0 = (uint64_t)tile << c_lg;
    for (uint32_t e = threadIdx.x; e < cnt; e += blockDim.x)
        lds[swz(e)] = A.Cc[((uint64_t)(e >> c_lg) << A.m2) + c0 + (e & cmask)];
    __syncthreads();
    inv_steps_to(lds, lg, lg - 3, c_lg, A.twi, threadIdx.x, blockDim.x);
    const uint32_t lgMp = lg - 3;
    const uint32_t ntask = (1u << lgMp) << c_lg;
    for (uint32_t task = threadIdx.x; task < ntask; task += blockDim.x) {
        const uint32_t q = task & cmask;
        const uint32_t n1 = task >> c_lg;
        uint64_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = lds[swz(((n1 + ((uint32_t)j << lgMp)) << c_lg) + q)];
        if (lg > 3) {
#pragma unroll
            for (int s = 1; s < 8; ++s) v[s] = fmul(v[s], A.twi[n1 * brev_small(s, 3)]);
        }
        dft_inv<8>(v);
#pragma unroll
        for (int j = 0; j < 8; ++j)
            A.Cc[((uint64_t)(n1 + ((uint32_t)j << lgMp)) << A.m2) + c0 + q] = v[j];
    }
}

// ------------------------------------------------------------------ carry scan

__device__ __forceinline__ CFn cf_id() { return CFn{CF_ID, CF_INF}; }

__device__ __forceinline__ CFn cf_limb(uint32_t t, uint32_t B) {
    uint32_t full = 1u << B;
    return CFn{t >> B, full - (t & (full - 1))};
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

struct ScanArgs {
    const uint32_t *t;   // digit sums: M regular limbs, then the top limb at index M if has_top
    uint32_t *out;       // normalised limbs
    uint64_t M;
    uint32_t B, has_top, s_top, dual;
    uint64_t ntiles;
    CFn *agg;
    uint32_t *tcarry;
    ScanResult *res;
};

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(ScanArgs A) {
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_PER_THREAD;
    CFn f = cf_id();
#pragma unroll
    for (int v = 0; v < SCAN_PER_THREAD; ++v) {
        uint64_t idx = base + v;
        if (idx < A.M) f = cf_compose(f, cf_limb(A.t[idx], A.B));
    }
    CFn excl, total;
    block_scan<SCAN_THREADS>(f, excl, total);
    if (threadIdx.x == 0) A.agg[blockIdx.x] = total;
}

// One workgroup: carry into every tile for global carry-in 0 (and 1 in dual
// mode), then the top limb and the selection of the dual variant.
__global__ __launch_bounds__(PREFIX_THREADS) void k_scan_prefix(ScanArgs A) {
    const uint64_t per = (A.ntiles + PREFIX_THREADS - 1) / PREFIX_THREADS;
    const uint64_t t0 = min((uint64_t)threadIdx.x * per, A.ntiles);
    const uint64_t t1 = min(t0 + per, A.ntiles);
    CFn f = cf_id();
    for (uint64_t j = t0; j < t1; ++j) f = cf_compose(f, A.agg[j]);
    CFn excl, total;
    block_scan<PREFIX_THREADS>(f, excl, total);
    const uint32_t nvar = A.dual ? 2u : 1u;
    for (uint32_t c = 0; c < nvar; ++c) {
        uint32_t carry = cf_eval(excl, c);
        for (uint64_t j = t0; j < t1; ++j) {
            A.tcarry[2 * j + c] = carry;
            carry = cf_eval(A.agg[j], carry);
        }
    }
    if (threadIdx.x == 0) {
        ScanResult r;
        r.final_carry = cf_eval(total, 0u);
        r.sel = 0u;
        r.carry_top[0] = r.carry_top[1] = 0u;
        r.ov[0] = r.ov[1] = 0u;
        r.pad[0] = r.pad[1] = 0u;
        if (A.has_top) {
            const uint32_t tt = A.t[A.M];
            for (uint32_t c = 0; c < 2; ++c) {
                uint32_t ct = cf_eval(total, c);
                uint32_t v = tt + ct;
                r.carry_top[c] = ct;
                r.ov[c] = v >> A.s_top;
            }
            r.sel = (A.dual && r.ov[1] != 0u) ? 1u : 0u;
            A.out[A.M] = (tt + r.carry_top[r.sel]) & ((1u << A.s_top) - 1);
        }
        *A.res = r;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(ScanArgs A) {
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_PER_THREAD;
    uint32_t tv[SCAN_PER_THREAD];
    CFn f = cf_id();
#pragma unroll
    for (int v = 0; v < SCAN_PER_THREAD; ++v) {
        uint64_t idx = base + v;
        tv[v] = idx < A.M ? A.t[idx] : 0u;
        if (idx < A.M) f = cf_compose(f, cf_limb(tv[v], A.B));
    }
    CFn excl, total;
    block_scan<SCAN_THREADS>(f, excl, total);
    const uint32_t sel = A.dual ? A.res->sel : 0u;
    uint32_t carry = cf_eval(excl, A.tcarry[2 * blockIdx.x + sel]);
    const uint32_t mask = (1u << A.B) - 1;
#pragma unroll
    for (int v = 0; v < SCAN_PER_THREAD; ++v) {
        uint64_t idx = base + v;
        if (idx < A.M) {
            uint32_t val = tv[v] + carry;
            A.out[idx] = val & mask;
            carry = val >> A.B;
        }
    }
}

// ------------------------------------------------------------------ fold / MH digits

// Digit sums of T = sum_{j<L} c_j 2^(Bj) + sum_{j>=L} c_j 2^(B(j-L)+e), which is
// S folded once at bit gamma (2^gamma = 1 mod p; e = BL - gamma).  Each
// coefficient is cut into B-bit pieces that land on consecutive digits.
__global__ void k_fold_gather(const uint64_t *__restrict__ c, uint32_t *t, uint64_t M, uint64_t L,
                              uint64_t N, uint32_t B, uint32_t e, uint32_t Q, uint32_t Q2) {
    uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const uint64_t mask = (1ull << B) - 1;
    uint64_t sum = 0;
    for (uint32_t q = 0; q < Q; ++q) {
        if (m >= q && m - q < L) sum += (c[m - q] >> (B * q)) & mask;
    }
    for (uint32_t q = 0; q < Q2; ++q) {
        if (m >= q) {
            uint64_t j = L + m - q;
            if (j < N) {
                unsigned __int128 v = (unsigned __int128)c[j] << e;
                sum += (uint64_t)(v >> (B * q)) & mask;
            }
        }
    }
    t[m] = (uint32_t)sum;
}

// Second fold: T = T_lo + 2^gamma V with T_lo = T mod 2^gamma; digits of
// T_lo + (V mod p) over L limbs (the top limb holds s_top bits).
__global__ void k_wrap_gather(const uint32_t *__restrict__ s, uint32_t *t, uint64_t L, uint64_t M,
                              uint32_t B, uint64_t gamma, uint32_t s_top) {
    uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= L) return;
    // V = bits [gamma, B*M) of the normalised T; it is below 2^66.
    unsigned __int128 V = 0;
    for (uint64_t idx = gamma / B; idx < M; ++idx) {
        uint64_t lo_bit = idx * B;
        unsigned __int128 limb = s[idx];
        if (lo_bit < gamma) V += limb >> (gamma - lo_bit);
        else if (lo_bit - gamma < 128) V += limb << (lo_bit - gamma);  // higher limbs are zero
    }
    if (gamma < 128) {
        const unsigned __int128 pm = (((unsigned __int128)1) << gamma) - 1;
        while (V >> gamma) V = (V & pm) + (V >> gamma);
        if (V == pm) V = 0;
    }
    uint32_t lo = (m + 1 < L) ? s[m] : (s[m] & ((1u << s_top) - 1));
    uint32_t vl = (B * m < 128) ? (uint32_t)((V >> (B * m)) & ((1ull << B) - 1)) : 0u;
    t[m] = lo + vl;
}

// MH digits: pieces of the product coefficients below limb L plus the limbs of
// c; everything at or above bit gamma is dropped later (mod 2^gamma).
__global__ void k_mh_gather(const uint64_t *__restrict__ cc, const uint64_t *__restrict__ cseed,
                            uint32_t *t, uint64_t L, uint32_t B, uint64_t gamma, uint32_t Q) {
    uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= L) return;
    const uint64_t mask = (1ull << B) - 1;
    uint64_t sum = bits_at(cseed, gamma, m * B, B);
    for (uint32_t q = 0; q < Q; ++q) {
        if (m >= q) sum += (cc[m - q] >> (B * q)) & mask;
    }
    t[m] = (uint32_t)sum;
}

// ------------------------------------------------------------------ output

__global__ void k_extract(const uint32_t *__restrict__ U, uint64_t *out, uint64_t out_words, uint64_t r,
                          uint64_t gamma, uint32_t B, const uint32_t *status) {
    uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= out_words || status[1] != 0u) return;
    uint64_t v = limbs_get64(U, B, gamma, gamma - r + 64 * w);
    uint64_t left = r - 64 * w;
    if (left < 64) v &= (1ull << left) - 1;
    out[w] = v;
}

__global__ void k_pack(const uint32_t *__restrict__ limbs, uint64_t *out, uint64_t words, uint64_t gamma,
                       uint32_t B, const uint32_t *status) {
    uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= words || status[1] != 0u) return;
    out[w] = limbs_get64(limbs, B, gamma, 64 * w);
}

__global__ void k_copy_status(const uint32_t *status, uint32_t *dst) { *dst = status[1]; }

inline unsigned blocks_for(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

hipError_t run_scan(pa_plan *p, const uint32_t *t, uint32_t *out, uint64_t M, bool top, bool dual,
                    hipStream_t st) {
    ScanArgs A;
    A.t = t;
    A.out = out;
    A.M = M;
    A.B = p->B;
    A.has_top = top ? 1u : 0u;
    A.s_top = p->s_top;
    A.dual = dual ? 1u : 0u;
    A.ntiles = (M + SCAN_TILE - 1) / SCAN_TILE;
    A.agg = p->agg;
    A.tcarry = p->tcarry;
    A.res = p->res;
    if (A.ntiles) hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)A.ntiles), dim3(SCAN_THREADS), 0, st, A);
    hipLaunchKernelGGL(k_scan_prefix, dim3(1), dim3(PREFIX_THREADS), 0, st, A);
    if (A.ntiles) hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)A.ntiles), dim3(SCAN_THREADS), 0, st, A);
    return hipGetLastError();
}

unsigned row_threads(const pa_plan *p) {
    unsigned n2 = 1u << p->m2;
    unsigned t = n2 / ROW_EPT;
    return t < 64 ? 64 : t;  // ROW_EPT elements per thread; N2 <= 8192 -> at most 512 threads
}

}  // namespace

namespace pa {

// Primitive 2^32-th root of unity r with r^(2^26) = 8, so that omega_64 = 8
// and the radix-8 twiddles are powers of two.  7 generates the
// multiplicative group of the field.
static uint64_t canonical_root_2_32() {
    const uint64_t r = gl_pow(7, (GL_P - 1) >> 32);
    const uint64_t w64 = gl_pow(r, 1ull << 26);
    uint64_t u = 0;
    for (uint64_t e = 1; e < 64; e += 2)
        if (gl_pow(8, e) == w64) {
            u = e;
            break;
        }
    uint64_t v = 1;
    while ((u * v) % 64 != 1) v += 2;  // u^-1 mod 64
    return gl_pow(r, v);
}

hipError_t launch_twiddles(pa_plan *p, hipStream_t st) {
    const uint64_t N = p->N;
    const uint64_t w = gl_pow(canonical_root_2_32(), 1ull << (32 - p->m));
    const uint64_t winv = gl_pow(w, N - 1);
    const uint64_t ninv = gl_pow(N % GL_P, GL_P - 2);
    const uint64_t w1 = gl_pow(w, 1ull << p->m2), w1i = gl_pow(winv, 1ull << p->m2);
    const uint64_t w2 = gl_pow(w, 1ull << p->m1), w2i = gl_pow(winv, 1ull << p->m1);
    const uint64_t n1 = 1ull << p->m1, n2 = 1ull << p->m2;
    hipLaunchKernelGGL(k_tw_pow, dim3(blocks_for(n1, 256)), dim3(256), 0, st, p->tw1f, n1, w1);
    hipLaunchKernelGGL(k_tw_pow, dim3(blocks_for(n1, 256)), dim3(256), 0, st, p->tw1i, n1, w1i);
    hipLaunchKernelGGL(k_tw_pow, dim3(blocks_for(n2, 256)), dim3(256), 0, st, p->tw2f, n2, w2);
    hipLaunchKernelGGL(k_tw_pow, dim3(blocks_for(n2, 256)), dim3(256), 0, st, p->tw2i, n2, w2i);
    hipLaunchKernelGGL(k_tw_four, dim3(blocks_for(N, 256)), dim3(256), 0, st, p->Wf, p->Wi, p->m1, p->m2,
                       w, winv, ninv);
    return hipGetLastError();
}

hipError_t launch_prologue(pa_plan *p, const uint64_t *a, const uint64_t *b, const uint64_t *c,
                           hipStream_t st) {
    phase_mark(p, PA_PH_PROLOGUE, true, st);
    hipLaunchKernelGGL(k_prologue, dim3(1), dim3(256), 0, st, a, b, c, p->k, p->W, p->gamma, p->notones,
                       p->status);
    phase_mark(p, PA_PH_PROLOGUE, false, st);
    return hipGetLastError();
}

hipError_t launch_mmh(pa_plan *p, const uint64_t *key, const uint64_t *a, hipStream_t st) {
    const unsigned ncol_tiles = 1u << (p->m2 - p->c_lg);
    const size_t col_lds = ((size_t)8 << p->m1) << p->c_lg;
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
    cf.c_lg = p->c_lg;
    cf.B = p->B;
    cf.s_top = p->s_top;
    cf.mode = 0;
    cf.key = key;
    cf.a = a;
    cf.b = nullptr;
    cf.ylimbs = nullptr;
    cf.notones = p->notones;
    cf.tw = p->tw1f;
    phase_mark(p, PA_PH_MMH_COL, true, st);
    hipLaunchKernelGGL(k_col_fwd, dim3(ncol_tiles, (unsigned)(2 * p->k)), dim3(COL_THREADS), col_lds, st, cf);
    phase_mark(p, PA_PH_MMH_COL, false, st);
    hipLaunchKernelGGL(k_status, dim3(1), dim3(256), 0, st, p->notones, p->k, p->status);

    RowArgs ra;
    ra.X = p->X;
    ra.N = p->N;
    ra.npairs = p->k;
    ra.a_off = p->k * p->N;
    ra.m2 = p->m2;
    ra.out = p->Cc;
    ra.Wf = p->Wf;
    ra.Wi = p->Wi;
    ra.twf = p->tw2f;
    ra.twi = p->tw2i;
    phase_mark(p, PA_PH_MMH_ROW, true, st);
    hipLaunchKernelGGL(k_row, dim3(1u << p->m1), dim3(row_threads(p)), (size_t)8 << p->m2, st, ra);
    phase_mark(p, PA_PH_MMH_ROW, false, st);

    ColInvArgs ci;
    ci.Cc = p->Cc;
    ci.m1 = p->m1;
    ci.m2 = p->m2;
    ci.c_lg = p->c_lg;
    ci.twi = p->tw1i;
    phase_mark(p, PA_PH_MMH_COLINV, true, st);
    hipLaunchKernelGGL(k_col_inv, dim3(ncol_tiles), dim3(COL_THREADS), col_lds, st, ci);
    phase_mark(p, PA_PH_MMH_COLINV, false, st);
    return hipGetLastError();
}

hipError_t launch_fold(pa_plan *p, hipStream_t st) {
    const uint32_t Q = (64 + p->B - 1) / p->B;
    const uint32_t Q2 = (64 + p->e_fold + p->B - 1) / p->B;
    phase_mark(p, PA_PH_FOLD, true, st);
    hipLaunchKernelGGL(k_fold_gather, dim3(blocks_for(p->M1, 256)), dim3(256), 0, st, p->Cc, p->t, p->M1,
                       p->L, p->N, p->B, p->e_fold, Q, Q2);
    hipError_t e = run_scan(p, p->t, p->s, p->M1, false, false, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wrap_gather, dim3(blocks_for(p->L, 256)), dim3(256), 0, st, p->s, p->t, p->L, p->M1,
                       p->B, p->gamma, p->s_top);
    e = run_scan(p, p->t, p->y, p->L - 1, true, true, st);
    phase_mark(p, PA_PH_FOLD, false, st);
    return e;
}

hipError_t launch_mh(pa_plan *p, const uint64_t *b, const uint64_t *c, hipStream_t st) {
    const unsigned ncol_tiles = 1u << (p->m2 - p->c_lg);
    const size_t col_lds = ((size_t)8 << p->m1) << p->c_lg;
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
    cf.c_lg = p->c_lg;
    cf.B = p->B;
    cf.s_top = p->s_top;
    cf.mode = 1;
    cf.key = nullptr;
    cf.a = nullptr;
    cf.b = b;
    cf.ylimbs = p->y;
    cf.notones = p->notones;
    cf.tw = p->tw1f;
    phase_mark(p, PA_PH_MH_COL, true, st);
    hipLaunchKernelGGL(k_col_fwd, dim3(ncol_tiles, 2u), dim3(COL_THREADS), col_lds, st, cf);
    phase_mark(p, PA_PH_MH_COL, false, st);

    RowArgs ra;
    ra.X = p->X;
    ra.N = p->N;
    ra.npairs = 1;
    ra.a_off = p->N;
    ra.m2 = p->m2;
    ra.out = p->Cc;
    ra.Wf = p->Wf;
    ra.Wi = p->Wi;
    ra.twf = p->tw2f;
    ra.twi = p->tw2i;
    phase_mark(p, PA_PH_MH_ROW, true, st);
    hipLaunchKernelGGL(k_row, dim3(1u << p->m1), dim3(row_threads(p)), (size_t)8 << p->m2, st, ra);
    phase_mark(p, PA_PH_MH_ROW, false, st);

    ColInvArgs ci;
    ci.Cc = p->Cc;
    ci.m1 = p->m1;
    ci.m2 = p->m2;
    ci.c_lg = p->c_lg;
    ci.twi = p->tw1i;
    phase_mark(p, PA_PH_MH_COLINV, true, st);
    hipLaunchKernelGGL(k_col_inv, dim3(ncol_tiles), dim3(COL_THREADS), col_lds, st, ci);
    phase_mark(p, PA_PH_MH_COLINV, false, st);

    const uint32_t Q = (64 + p->B - 1) / p->B;
    phase_mark(p, PA_PH_MH_CARRY, true, st);
    hipLaunchKernelGGL(k_mh_gather, dim3(blocks_for(p->L, 256)), dim3(256), 0, st, p->Cc, c, p->t, p->L, p->B,
                       p->gamma, Q);
    hipError_t e = run_scan(p, p->t, p->U, p->L - 1, true, false, st);
    phase_mark(p, PA_PH_MH_CARRY, false, st);
    return e;
}

hipError_t launch_finish(pa_plan *p, uint64_t *out, uint32_t *d_status, uint64_t *y_out, uint64_t *U_out,
                         hipStream_t st) {
    phase_mark(p, PA_PH_FINISH, true, st);
    hipLaunchKernelGGL(k_extract, dim3(blocks_for(p->out_words, 256)), dim3(256), 0, st, p->U, out,
                       p->out_words, p->r, p->gamma, p->B, p->status);
    if (y_out)
        hipLaunchKernelGGL(k_pack, dim3(blocks_for(p->W, 256)), dim3(256), 0, st, p->y, y_out, p->W, p->gamma,
                           p->B, p->status);
    if (U_out)
        hipLaunchKernelGGL(k_pack, dim3(blocks_for(p->W, 256)), dim3(256), 0, st, p->U, U_out, p->W, p->gamma,
                           p->B, p->status);
    hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(1), 0, st, p->status, d_status ? d_status : p->status_out);
    phase_mark(p, PA_PH_FINISH, false, st);
    return hipGetLastError();
}

}  // namespace pa
