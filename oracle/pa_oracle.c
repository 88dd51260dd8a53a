/*
 * Plain CPU oracle for the MMH-MH privacy-amplification hash.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library; the product path never
 * does.  It shares no code, header or table with the GPU library.
 *
 * What it computes (Yan, Li, Mao, Chen, arXiv 2105.13678):
 *   split   x_i = key bits [i*gamma, (i+1)*gamma), zero past n   (Alg. 1, split)
 *   reload  any x_i == 2^gamma - 1  ->  status RELOAD, no output  (Sec. 3.1, Alg. 1)
 *   MMH     y = (sum_i a_i x_i) mod p,  p = 2^gamma - 1            (Sec. 2.1 eq. 2)
 *   MH      z = ((b y + c) mod 2^gamma) >> (gamma - r)             (Sec. 2.2 eq. 4)
 * with gamma the smallest Mersenne exponent above r (Sec. 4, Table 3) unless
 * the caller names one, and k = ceil(n / gamma).
 *
 * Arithmetic: big integers as little-endian arrays of 64-bit words; products by
 * schoolbook multiplication below a cut-off and Karatsuba's split above it;
 * the sum is formed exactly and reduced mod 2^gamma - 1 by repeated folding
 * (x mod M = floor(x / 2^gamma) + x mod 2^gamma, Sec. 3.1) until it is below
 * 2^gamma, then p itself maps to 0.  No step is fused or reordered beyond that.
 *
 * Status codes and precedence match the library's interface: SEED_RANGE (-6)
 * if any seed word has bits >= gamma set, else SEED_B_EVEN (-5) if b is even,
 * else RELOAD (2) if some chunk is all ones, else OK (0).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef unsigned __int128 u128;

static const u64 MERSENNE[] = {
    2, 3, 5, 7, 13, 17, 19, 31, 61, 89, 107, 127, 521, 607, 1279, 2203, 2281,
    3217, 4253, 4423, 9689, 9941, 11213, 19937, 21701, 23209, 44497, 86243,
    110503, 132049, 216091, 756839, 859433, 1257787, 1398269, 2976221, 3021377,
    6972593, 13466917, 20996011, 24036583, 25964951, 30402457, 32582657,
    37156667, 42643801, 43112609, 57885161, 74207281, 77232917, 82589933,
    136279841};
#define N_MERSENNE (sizeof(MERSENNE) / sizeof(MERSENNE[0]))

enum { O_OK = 0, O_RELOAD = 2, O_ERR_ARG = -1, O_ERR_NO_GAMMA = -2, O_ERR_GAMMA = -3,
       O_ERR_NOMEM = -7, O_ERR_SEED_B_EVEN = -5, O_ERR_SEED_RANGE = -6 };

int oracle_plan(u64 n, u64 r, u64 gamma_req, u64 *gamma, u64 *k) {
    if (n < 2 || r < 1 || r >= n) return O_ERR_ARG;
    u64 g = 0;
    if (gamma_req == 0) {
        for (size_t i = 0; i < N_MERSENNE; i++)
            if (MERSENNE[i] > r) { g = MERSENNE[i]; break; }
        if (!g) return O_ERR_NO_GAMMA;
    } else {
        int found = 0;
        for (size_t i = 0; i < N_MERSENNE; i++) found |= (MERSENNE[i] == gamma_req);
        if (!found || gamma_req <= r) return O_ERR_GAMMA;
        g = gamma_req;
    }
    *gamma = g;
    *k = (n + g - 1) / g;
    return O_OK;
}

/* ---------- word-array helpers ---------- */

/* dst[0..nw) = bits [off, off+len) of src; bits at positions >= valid read as 0.
 * src holds ceil(valid/64) words. */
static void extract_bits(const u64 *src, u64 valid, u64 off, u64 len, u64 *dst, size_t nw) {
    memset(dst, 0, nw * sizeof(u64));
    u64 lim = off + len < valid ? off + len : valid;
    if (off >= lim) return;
    u64 cnt = lim - off;
    u64 nsrc = (valid + 63) / 64;
    for (u64 i = 0; i * 64 < cnt; i++) {
        u64 p = off + i * 64;
        u64 w = p >> 6, s = p & 63;
        u64 v = src[w] >> s;
        if (s && w + 1 < nsrc) v |= src[w + 1] << (64 - s);
        u64 take = cnt - i * 64;
        if (take < 64) v &= (((u64)1) << take) - 1;
        dst[i] = v;
    }
}

static int is_zero(const u64 *a, size_t n) {
    for (size_t i = 0; i < n; i++)
        if (a[i]) return 0;
    return 1;
}

/* a[0..na) += b[0..nb), returns carry out of a[na-1]; na >= nb */
static u64 add_into(u64 *a, size_t na, const u64 *b, size_t nb) {
    u64 carry = 0;
    for (size_t i = 0; i < na; i++) {
        u64 bi = i < nb ? b[i] : 0;
        if (i >= nb && !carry) break;
        u128 s = (u128)a[i] + bi + carry;
        a[i] = (u64)s;
        carry = (u64)(s >> 64);
    }
    return carry;
}

/* a[0..na) -= b[0..nb), nb <= na, value of a >= value of b */
static void sub_ext(u64 *a, size_t na, const u64 *b, size_t nb) {
    u64 borrow = 0;
    for (size_t i = 0; i < na; i++) {
        u64 bi = i < nb ? b[i] : 0;
        if (i >= nb && !borrow) break;
        u64 t = a[i] - bi;
        u64 b1 = a[i] < bi;
        u64 t2 = t - borrow;
        u64 b2 = t < borrow;
        a[i] = t2;
        borrow = b1 | b2;
    }
}

/* ---------- multiplication ---------- */

/* out[0..na+nb) = a * b, schoolbook */
static void mul_school(const u64 *a, size_t na, const u64 *b, size_t nb, u64 *out) {
    memset(out, 0, (na + nb) * sizeof(u64));
    for (size_t i = 0; i < na; i++) {
        u64 carry = 0;
        u64 ai = a[i];
        if (!ai) continue;
        for (size_t j = 0; j < nb; j++) {
            u128 t = (u128)ai * b[j] + out[i + j] + carry;
            out[i + j] = (u64)t;
            carry = (u64)(t >> 64);
        }
        out[i + nb] = carry;
    }
}

#define KARA_CUTOFF 32

/* out[0..2n) = a[0..n) * b[0..n); scratch needs kara_scratch(n) words */
static size_t kara_scratch(size_t n) {
    if (n < KARA_CUTOFF) return 0;
    size_t h = n / 2, m = n - h + 1;
    return 4 * m + kara_scratch(m);
}

static void kara(const u64 *a, const u64 *b, size_t n, u64 *out, u64 *scratch) {
    if (n < KARA_CUTOFF) {
        mul_school(a, n, b, n, out);
        return;
    }
    size_t h = n / 2;        /* low half length */
    size_t hn = n - h;       /* high half length (>= h) */
    size_t m = hn + 1;       /* length of a0+a1 and b0+b1 with room for a carry */
    u64 *sa = scratch, *sb = scratch + m, *z1 = scratch + 2 * m, *rest = scratch + 4 * m;

    /* z0 = a0*b0 into out[0..2h), z2 = a1*b1 into out[2h..2n) */
    kara(a, b, h, out, rest);
    kara(a + h, b + h, hn, out + 2 * h, rest);

    /* sa = a0 + a1, sb = b0 + b1 (m words, a0 zero-extended) */
    memset(sa, 0, m * sizeof(u64));
    memset(sb, 0, m * sizeof(u64));
    memcpy(sa, a + h, hn * sizeof(u64));
    memcpy(sb, b + h, hn * sizeof(u64));
    add_into(sa, m, a, h);
    add_into(sb, m, b, h);

    /* z1 = sa*sb - z0 - z2 = a0*b1 + a1*b0 (2m words) */
    kara(sa, sb, m, z1, rest);
    sub_ext(z1, 2 * m, out, 2 * h);
    sub_ext(z1, 2 * m, out + 2 * h, 2 * hn);
    /* out += z1 << (64*h); z1 < 2^(128*hn+...) fits in out[h..2n) */
    size_t span = 2 * n - h;
    size_t zl = 2 * m;
    while (zl > 0 && z1[zl - 1] == 0) zl--;
    if (zl > span) zl = span; /* high words beyond the product are zero */
    add_into(out + h, span, z1, zl);
}

/* out[0..2n) = a[0..n) * b[0..n) */
static int mul_equal(const u64 *a, const u64 *b, size_t n, u64 *out) {
    size_t s = kara_scratch(n);
    u64 *scratch = s ? (u64 *)malloc(s * sizeof(u64)) : NULL;
    if (s && !scratch) return -1;
    kara(a, b, n, out, scratch);
    free(scratch);
    return 0;
}

/* ---------- the hash ---------- */

/* Reduce v[0..nv) modulo 2^gamma - 1 in place; result in v[0..W), canonical. */
static void mod_mersenne(u64 *v, size_t nv, u64 gamma, size_t W) {
    u64 *hi = (u64 *)calloc(nv + 1, sizeof(u64));
    u64 top_bits = gamma % 64;
    for (;;) {
        /* hi = v >> gamma */
        size_t nh = 0;
        u64 total_bits = (u64)nv * 64;
        if (total_bits > gamma) {
            u64 hb = total_bits - gamma;
            nh = (size_t)((hb + 63) / 64);
            extract_bits(v, total_bits, gamma, hb, hi, nh);
        }
        if (is_zero(hi, nh)) break;
        /* v = v mod 2^gamma */
        for (size_t i = W; i < nv; i++) v[i] = 0;
        if (top_bits) v[W - 1] &= (((u64)1) << top_bits) - 1;
        /* v += hi */
        add_into(v, nv, hi, nh < nv ? nh : nv);
    }
    free(hi);
    /* now v < 2^gamma; p = 2^gamma - 1 maps to 0 */
    int all_ones = 1;
    for (size_t i = 0; i < W; i++) {
        u64 want = (i == W - 1 && top_bits) ? ((((u64)1) << top_bits) - 1) : ~(u64)0;
        if (v[i] != want) { all_ones = 0; break; }
    }
    if (all_ones) memset(v, 0, W * sizeof(u64));
}

/* The terms a_i x_i of the MMH sum (Sec. 2.1 eq. 2) for i in [i0, i1), added
 * into S (ns words).  Integer addition is exact and associative, so partial
 * sums over disjoint ranges of i add up to the same S. */
struct partial_sum {
    const u64 *key, *a;
    u64 n, g, i0, i1;
    size_t W, ns;
    u64 *S;
    int err;
};

static void *add_terms(void *arg) {
    struct partial_sum *P = (struct partial_sum *)arg;
    u64 *x = (u64 *)calloc(P->W, sizeof(u64));
    u64 *prod = (u64 *)calloc(2 * P->W, sizeof(u64));
    if (!x || !prod) P->err = 1;
    for (u64 i = P->i0; i < P->i1 && !P->err; i++) {
        extract_bits(P->key, P->n, i * P->g, P->g, x, P->W);
        if (mul_equal(P->a + i * P->W, x, P->W, prod)) { P->err = 1; break; }
        add_into(P->S, P->ns, prod, 2 * P->W);
    }
    free(x);
    free(prod);
    return NULL;
}

static int hash_impl(const u64 *key, u64 n, u64 r, u64 gamma, const u64 *a, const u64 *b, const u64 *c,
                     u64 *out, u64 *y_out, u64 *U_out, int nthreads);

/*
 * Full hash.  key: ceil(n/64) words; a: k*W words; b, c: W words, W = ceil(gamma/64);
 * out: ceil(r/64) words.  y_out and U_out (W words each, may be NULL) receive
 * the MMH value y and the MH value before truncation, U.
 */
int oracle_hash(const u64 *key, u64 n, u64 r, u64 gamma, const u64 *a, const u64 *b,
                const u64 *c, u64 *out, u64 *y_out, u64 *U_out) {
    return hash_impl(key, n, r, gamma, a, b, c, out, y_out, U_out, 1);
}

/* The same with the k products of the MMH sum spread over up to `nthreads`
 * threads (contiguous ranges of i, each summed apart, then the partial sums
 * added); every other step as in oracle_hash.  For timing on several cores. */
int oracle_hash_threads(const u64 *key, u64 n, u64 r, u64 gamma, const u64 *a, const u64 *b,
                        const u64 *c, u64 *out, u64 *y_out, u64 *U_out, int nthreads) {
    return hash_impl(key, n, r, gamma, a, b, c, out, y_out, U_out, nthreads < 1 ? 1 : nthreads);
}

static int hash_impl(const u64 *key, u64 n, u64 r, u64 gamma, const u64 *a, const u64 *b, const u64 *c,
                     u64 *out, u64 *y_out, u64 *U_out, int nthreads) {
    u64 g, k;
    int st = oracle_plan(n, r, gamma, &g, &k);
    if (st) return st;
    size_t W = (size_t)((g + 63) / 64);
    u64 top_bits = g % 64;
    u64 top_mask = top_bits ? ((((u64)1) << top_bits) - 1) : ~(u64)0;

    /* seed checks */
    for (u64 i = 0; i < k; i++)
        if (a[i * W + W - 1] & ~top_mask) return O_ERR_SEED_RANGE;
    if ((b[W - 1] & ~top_mask) || (c[W - 1] & ~top_mask)) return O_ERR_SEED_RANGE;
    if ((b[0] & 1) == 0) return O_ERR_SEED_B_EVEN;

    u64 *x = (u64 *)calloc(W, sizeof(u64));
    u64 *prod = (u64 *)calloc(2 * W, sizeof(u64));
    size_t ns = 2 * W + 2;
    u64 *S = (u64 *)calloc(ns, sizeof(u64));
    if (!x || !prod || !S) { free(x); free(prod); free(S); return O_ERR_NOMEM; }

    /* reload check on every chunk before any output (Alg. 1) */
    for (u64 i = 0; i < k; i++) {
        extract_bits(key, n, i * g, g, x, W);
        int all_ones = 1;
        for (size_t w = 0; w < W; w++) {
            u64 want = (w == W - 1) ? top_mask : ~(u64)0;
            if (x[w] != want) { all_ones = 0; break; }
        }
        if (all_ones) { free(x); free(prod); free(S); return O_RELOAD; }
    }

    /* S = sum_i a_i x_i, exact: T contiguous ranges of i, one partial sum each */
    u64 T = (u64)nthreads < k ? (u64)nthreads : k;
    struct partial_sum *parts = (struct partial_sum *)calloc(T, sizeof(struct partial_sum));
    pthread_t *tid = (pthread_t *)calloc(T, sizeof(pthread_t));
    int bad = !parts || !tid;
    for (u64 t = 0; t < T && !bad; t++) {
        struct partial_sum *P = &parts[t];
        P->key = key;
        P->a = a;
        P->n = n;
        P->g = g;
        P->i0 = k * t / T;
        P->i1 = k * (t + 1) / T;
        P->W = W;
        P->ns = ns;
        P->S = t == 0 ? S : (u64 *)calloc(ns, sizeof(u64));
        if (!P->S) bad = 1;
    }
    u64 started = 0; /* threads 1..started were created */
    for (u64 t = 1; t < T && !bad; t++) {
        if (pthread_create(&tid[t], NULL, add_terms, &parts[t]))
            bad = 1;
        else
            started = t;
    }
    if (!bad) add_terms(&parts[0]);
    for (u64 t = 1; t <= started; t++) pthread_join(tid[t], NULL);
    for (u64 t = 0; t < T && parts; t++) {
        bad |= parts[t].err;
        if (t > 0 && parts[t].S) {
            if (!bad) add_into(S, ns, parts[t].S, ns);
            free(parts[t].S);
        }
    }
    free(parts);
    free(tid);
    if (bad) { free(x); free(prod); free(S); return O_ERR_NOMEM; }
    /* y = S mod p */
    mod_mersenne(S, ns, g, W);
    if (y_out) memcpy(y_out, S, W * sizeof(u64));

    /* U = (b*y + c) mod 2^gamma */
    if (mul_equal(b, S, W, prod)) { free(x); free(prod); free(S); return O_ERR_NOMEM; }
    add_into(prod, 2 * W, c, W);
    for (size_t i = W; i < 2 * W; i++) prod[i] = 0;
    prod[W - 1] &= top_mask;
    if (U_out) memcpy(U_out, prod, W * sizeof(u64));

    /* z = U >> (gamma - r), r bits */
    size_t nout = (size_t)((r + 63) / 64);
    extract_bits(prod, g, g - r, r, out, nout);

    free(x);
    free(prod);
    free(S);
    return O_OK;
}

/* Product of two equal-length word arrays, exposed for tests. */
int oracle_mul(const u64 *a, const u64 *b, u64 n, u64 *out) { return mul_equal(a, b, (size_t)n, out); }
