// Internal declarations shared by the libpa translation units.
//
// Arithmetic: exact convolutions of B-bit limb sequences by number-theoretic
// transforms of length N = 2^m or N = 3 * 2^m modulo three primes below 2^30
// (4p < 2^32 lets the transforms keep residues only partially reduced).  The
// primes are the three largest below 2^30 with N | p - 1, from a fixed table
// per length.
// A gamma-bit number is cut into L = ceil(gamma/B) limbs (the paper's 2^B-ary
// words); every coefficient of the sum of the k limb convolutions is at most
// k*L*(2^B-1)^2, which the plan checks is below p0*p1*p2, so the
// Chinese-remainder reconstruction of the three transforms is the exact
// integer coefficient.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "pa.h"

namespace pa {

constexpr int NPRIMES = 3;
constexpr uint32_t MAX_LOG2N = 24;      // longest power-of-two transform with three such primes
constexpr uint32_t MAX_LOG2N_MIX = 23;  // longest transform 3 * 2^m
constexpr uint32_t MAX_LOG2N_MIX5 = 20; // longest transform 5 * 2^m (column passes of at most 256 rows)

// Length forms: mix 0 for N = 2^m, 1 for N = 3 * 2^m, 2 for N = 5 * 2^m.
constexpr uint32_t len_factor_of(uint32_t mix) { return mix == 2 ? 5u : mix == 1 ? 3u : 1u; }

// The three largest primes p < 2^30 with 2^max_lg | p - 1 (product 2^log2P),
// for the transform lengths 2^m, m <= max_lg, not served by an earlier row.
struct PrimeTriple {
    uint32_t max_lg;
    uint32_t p[NPRIMES];
};
constexpr PrimeTriple PRIME_TRIPLES[] = {
    {20, {1053818881u, 1051721729u, 1045430273u}},  // 2^89.905
    {21, {1012924417u, 1004535809u, 998244353u}},   // 2^89.715
    {22, {998244353u, 985661441u, 943718401u}},     // 2^89.585
    {23, {998244353u, 897581057u, 880803841u}},     // 2^89.351
    {24, {754974721u, 469762049u, 167772161u}},     // 2^85.621
};
// The same for the lengths 3 * 2^m: the three largest primes p < 2^30 with
// 3 * 2^max_lg | p - 1.
constexpr PrimeTriple PRIME_TRIPLES_3[] = {
    {18, {1073479681u, 1062469633u, 1056178177u}},  // 2^89.961
    {19, {1053818881u, 1049100289u, 1012924417u}},  // 2^89.855
    {20, {1053818881u, 1012924417u, 975175681u}},   // 2^89.750
    {21, {1012924417u, 975175681u, 962592769u}},    // 2^89.619
    {22, {943718401u, 918552577u, 880803841u}},     // 2^89.303
    {23, {880803841u, 754974721u, 377487361u}},     // 2^87.698
};
// The same for the lengths 5 * 2^m: the three largest primes p < 2^30 with
// 5 * 2^max_lg | p - 1.
constexpr PrimeTriple PRIME_TRIPLES_5[] = {
    {18, {1073479681u, 1068236801u, 1056440321u}},  // 2^89.969
    {19, {1056440321u, 1053818881u, 985661441u}},   // 2^89.826
    {20, {1053818881u, 985661441u, 975175681u}},    // 2^89.711
};

// Per-prime constants (Montgomery form x*2^32 mod p where noted).
struct PrimeConst {
    uint32_t p;
    uint32_t pinv;   // -p^-1 mod 2^32
    uint32_t one;    // 2^32 mod p (1 in Montgomery form)
    uint32_t p2;     // 2p
    uint32_t w16[8];   // omega_16^j, j < 8, Montgomery form
    uint32_t w16i[8];  // omega_16^-j, j < 8, Montgomery form
};

struct PrimeSet {
    PrimeConst c[NPRIMES];
};

// Constants for the Chinese-remainder (Garner) reconstruction.
struct CrtConst {
    uint32_t inv_p0_mod_p1;     // p0^-1 mod p1, Montgomery form (mod p1)
    uint32_t one_sub;           // 1 when p0, p1 < 2 p2 and p0 < 2 p1: a conditional subtraction reduces
    uint32_t inv_p0p1_mod_p2;   // (p0 p1)^-1 mod p2, Montgomery form (mod p2)
    uint32_t inv_p1_mod_p2;     // p1^-1 mod p2, Montgomery form (mod p2)
    uint64_t p0p1;              // p0 * p1
};

// Inverse radix-3 step of the lengths N = 3 * 2^m (Montgomery form, per
// prime): with w = omega_3 = omega_N^(N/3), the outputs s0 + w^-n0 u1 +
// w^-2n0 u2 (n0 = 1, 2) are s0 - (u1 + u2)/2 +- h (u1 - u2), h = (w^-1 - w^-2)/2.
struct Mix3Const {
    uint32_t neg_half[NPRIMES];  // -1/2 mod p
    uint32_t h[NPRIMES];
};

// Inverse radix-5 step of the lengths N = 5 * 2^m: omega_5^-e (omega_5 =
// omega_N^(N/5)) for e < 5, Montgomery form, per prime.
struct Mix5Const {
    uint32_t wi[NPRIMES][5];
};

// ---------------------------------------------------------------- carry functions
// Carry transfer function of a run of limbs: carry_out = g + [carry_in >= th].
// th == CF_INF means the run's carry out does not depend on its carry in;
// g == CF_ID marks the identity (an empty run).
struct CFn {
    uint32_t g, th;
};
constexpr uint32_t CF_INF = 0xFFFFFFFFu;
constexpr uint32_t CF_ID = 0xFFFFFFFFu;

constexpr int SCAN_THREADS = 256;
constexpr int CARRY_PER_THREAD = 4;                          // consecutive digits per thread
constexpr int CARRY_TILE = SCAN_THREADS * CARRY_PER_THREAD;  // digits per workgroup and per aggregate
constexpr uint32_t R16_TW = 16 * 256 + 16 * 16;  // words per prime of the row-kernel step-twiddle table

// Steps of the per-block launch sequence.  The batched path records each
// block's launches with their step and runs every step of all blocks as
// multi-block launches, in this order.
enum Step : int {
    SP_MMH_COL = 0,
    SP_MMH_ROW,
    SP_MMH_COLINV,
    SP_FOLD_CRT3,
    SP_FOLD_DIGIT,
    SP_FOLD_APPLY,
    SP_FOLD_WRAP,
    SP_MH_COL,
    SP_MH_ROW,
    SP_MH_COLINV,
    SP_MH_CRT3,
    SP_MH_DIGIT,
    SP_MH_APPLY,
    SP_COUNT
};

// One recorded kernel launch of one block: the kernel in its single-block
// form (which identifies the instance) and its multi-block form (arguments:
// a table of argument structs, the blocks' grid placement, the owner table),
// the block's grid, the workgroup size and dynamic LDS, and the argument
// struct by value.
constexpr uint32_t KARGS_MAX = 512;
struct KLaunch {
    int step;
    const void *single, *multi;
    dim3 grid, block;
    uint32_t lds;
    uint32_t args_size;
    alignas(16) unsigned char args[KARGS_MAX];
};

// Device status flag bits (written by the fold's reconstruction kernel).
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
    uint32_t mix;               // length form: 0: N = 2^m; 1: N = 3 * 2^m, 2: N = 5 * 2^m (a radix-3 or
                                // radix-5 step over three or five length-2^m transforms)
    uint32_t rf;                // N / 2^m: 1, 3 or 5
    uint64_t Nsub;              // 2^m: length of the power-of-two transforms
    uint32_t m, m1, m2;         // 2^m = 2^m1 (column length) * 2^m2 (row length)
    uint32_t c_lg, c_lg_mh;     // 2^c columns per tile of the forward column pass: key chunks and seeds; MH stage
    uint32_t ci_lg;             // columns per tile of the inverse column pass
    uint32_t s_top;             // bits in the top limb: gamma - B*(L-1), in [1, B]
    uint32_t e_fold;            // B*L - gamma, in [0, B)
    uint64_t M1;                // digit count of the folded sum before reduction
    uint64_t ntiles_max;
    double exact_log2;
    pa::PrimeSet primes;
    pa::CrtConst crt;
    pa::Mix3Const mix3;
    pa::Mix5Const mix5;

    // device memory (one allocation, carved)
    void *base;
    size_t workspace_bytes;
    size_t scratch_bytes;  // [base, base + scratch_bytes): everything but the twiddle tables
    uint32_t *X;        // 2k arrays x 3 primes x N words: column-pass outputs of x_i (0..k-1), a_i (k..2k-1)
    uint32_t *Cc;       // 3 x N words: convolution residues
    uint64_t *t;        // digit sums (max(M1, L) + pad)
    uint32_t *s;        // normalised limbs of the folded sum (M1)
    uint32_t *y;        // MMH output limbs (L)
    uint32_t *U;        // MH value limbs (L)
    uint32_t *C96;      // N = 3 * 2^m only: 3 x N words, reconstructed coefficients as word planes
                        // (bits 0-31, 32-63, 64-95); for N = 2^m the digit kernels reconstruct them
    pa::CFn *agg;       // carry functions of CARRY_TILE-digit tiles
    pa::CFn *agg_w;     // the same for the wrap chain (second fold)
    uint32_t *tflags;   // per first-fold tile: its limbs in [min(32, L - 1), L) all ones
    uint32_t *notones;  // k x 2^m2 words: tile x of key chunk i saw a limb that is not all ones (i * tiles + x)
    uint32_t *status;   // seed/reload flags
    uint32_t *status_out;  // final flags of the last call (pa_hash reads it back)
    uint32_t *tw1f, *tw1i;  // per prime: omega_{N1}^+-j, j < N1 (Montgomery form)
    uint32_t *tw2f, *tw2i;  // per prime: omega_{N2}^+-j, j < N2
    uint32_t *Wf, *Wi;      // per prime: four-step twiddles, stored (bit-reversed) row order
    uint32_t *R16f, *R16i;  // per prime: step twiddles of the 4096-point row kernel in thread order
                            // (R16_TW words: [j][t] omega^(t brev(j)), then [j][n1] omega^(16 n1 brev(j)))
    uint32_t *G3;           // N = 3 * 2^m only: three tables of NPRIMES x 3 x N1 words, entry
                            // [q][k0][r] = omega_N^(k0 r N2), omega_N^(k0 (r N2 + N/3)), omega_N^(-k0 r N2)
    const uint32_t *res_a;  // resident seed transforms (k x 3 x N words) or null
    const uint32_t *res_b;  // resident transform of b (3 x N words) or null
    uint32_t *h_status;     // pinned host word
    std::vector<pa::KLaunch> *rec;  // non-null: record the hash's launches here instead of launching

    // phase profiling (pa_plan_set_profiling)
    uint32_t profiling;  // phase mask
    struct EvPair {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<EvPair> *pending;
    std::vector<hipEvent_t> *event_pool;
};

namespace pa {

// Offsets (bytes) of a plan's device buffers: the per-call scratch occupies
// [0, scratch_bytes), the read-only twiddle tables (which depend only on the
// transform length) the following table_bytes.
struct PlanLayout {
    size_t oX, oC, oC96, oT, oS, oY, oU, oAgg, oNo, oSt, oSo, oTf;
    size_t oT1, oT2, oW, oR16, oG3;
    size_t scratch_bytes, table_bytes, total;
};

// Makes `dev` the current HIP device for a scope and restores the previous
// one on exit (the entry points may be called with another device current).
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    DeviceGuard(const DeviceGuard &) = delete;
    DeviceGuard &operator=(const DeviceGuard &) = delete;
};

// Identifies a plan's transform length (and so its primes and twiddle tables).
inline uint32_t len_key(const pa_plan &p) { return p.rf << 7 | p.m; }

// Host-side plan derivation (no device access) and buffer binding (pa_api.cpp).
pa_status derive_plan(const pa_params *prm, pa_plan *p, PlanLayout *lay);
void bind_scratch(pa_plan *p, void *scratch, const PlanLayout &lay);
void bind_tables(pa_plan *p, void *tables, const PlanLayout &lay);
// Enqueue one complete hash on `st` (no synchronisation).
pa_status enqueue_hash(pa_plan *p, const uint64_t *key, const uint64_t *a, const uint64_t *b,
                       const uint64_t *c, uint64_t *out, uint32_t *d_status, uint64_t *y_out,
                       uint64_t *U_out, hipStream_t st);

// Host-side constant setup (pa_kernels.hip): Montgomery constants, small
// roots and CRT constants for the three primes of the plan's triple.
void init_prime_constants(pa_plan *p, const uint32_t primes[NPRIMES]);

// Kernel launchers (pa_kernels.hip).  All enqueue on `st` and return the
// first HIP error seen.
// With hdr (a device word): skip the build when *hdr == want, else build and
// then set *hdr = want (tables kept in memory that outlives one call).
hipError_t launch_twiddles(pa_plan *p, hipStream_t st, uint32_t *hdr = nullptr, uint32_t want = 0);
hipError_t launch_mmh(pa_plan *p, const uint64_t *key, const uint64_t *a, hipStream_t st);
// The seeds of a hash call (device words), for the status checks of the fold.
struct Seeds {
    const uint64_t *a, *b, *c;
};
hipError_t launch_fold(pa_plan *p, const Seeds &seeds, hipStream_t st);
// The second fold's general case (a no-op unless the first fold flagged it):
// recomputes y.  launch_fold runs it unless wrap_inline(p); with the inline
// form the MH stage corrects for the rare case itself and y is recomputed
// only where y is an output (pa_hash_stages), after the MH stage.
bool wrap_inline(const pa_plan *p);
hipError_t launch_wrap(pa_plan *p, hipStream_t st);
// The MH stage ends with the output extraction (z into out, flags into d_status,
// or the plan's own status word when d_status is null).
hipError_t launch_mh(pa_plan *p, const uint64_t *b, const uint64_t *c, uint64_t *out, uint32_t *d_status,
                     hipStream_t st);
// Stage values for pa_hash_stages (y, U packed into words; nullptr skips).
hipError_t launch_finish(pa_plan *p, uint64_t *y_out, uint64_t *U_out, hipStream_t st);
// Fills `count` words at dst with `word` (pa_plan_fill_scratch).
hipError_t launch_fill(uint32_t *dst, uint64_t count, uint32_t word, hipStream_t st);
hipError_t launch_seed_transforms(pa_plan *p, const uint64_t *a, uint64_t kmax, const uint64_t *b,
                                  uint32_t *dst_a, uint32_t *dst_b, hipStream_t st);

// Marks the start or end of a phase on `st` when profiling is on (pa_api.cpp).
void phase_mark(pa_plan *p, int phase, bool begin, hipStream_t st);

}  // namespace pa
