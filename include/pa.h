/*
 * pa.h -- C interface of libpa, the MI355X (gfx950) implementation of the
 * MMH-MH privacy-amplification hash of Yan, Li, Mao and Chen, "An efficient
 * hybrid hash based privacy amplification algorithm for quantum key
 * distribution" (arXiv 2105.13678).
 *
 * The hash (Algorithm 1, with MMH from Sec. 2.1 eq. (2) and MH from Sec. 2.2
 * eq. (4)):
 *
 *   inputs   key x of n bits; output length r (the paper's beta)
 *   plan     gamma = Mersenne exponent with gamma > r; p = 2^gamma - 1;
 *            k = ceil(n / gamma)                       (Sec. 4, Table 3)
 *   split    x_i = key bits [i*gamma, (i+1)*gamma), zero past bit n
 *   reload   some x_i == 2^gamma - 1  ->  PA_RELOAD, nothing written
 *   MMH      y = (sum_{i<k} a_i x_i) mod p, canonical in [0, p)
 *   MH       U = (b*y + c) mod 2^gamma;   z = U >> (gamma - r)
 *
 * Bit order is little-endian everywhere: key bit j is bit (j mod 64) of word
 * j/64; bit t of chunk x_i is key bit i*gamma + t; bit t of the output z is
 * bit gamma - r + t of U.
 *
 * All buffers passed to the hash entry points are DEVICE pointers on the
 * plan's device, owned by the caller, and must stay valid until the call has
 * completed on its stream.  Layouts (all uint64_t little-endian words):
 *   key : ceil(n/64) words; bits >= n of the last word are ignored
 *   a   : k chunks of W = ceil(gamma/64) words, chunk i at a + i*W
 *   b, c: W words each; b must be odd
 *   out : ceil(r/64) words; bits >= r of the last word are written as 0
 * Every seed word must have its bits >= gamma (within its chunk) clear.
 *
 * Errors are return codes; nothing is thrown across this interface.  Errors
 * the host can see (arguments, plan shape) return before any launch.
 * Conditions found on the device (RELOAD, SEED_B_EVEN, SEED_RANGE) come back
 * through a status word; on any status other than PA_OK the output buffer is
 * left untouched.  A plan must be used by one host thread at a time.
 */
#ifndef PA_H
#define PA_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pa_status {
    PA_OK = 0,
    PA_PENDING = 1,          /* request not finished yet (pa_poll)                       */
    PA_RELOAD = 2,           /* a key chunk equals 2^gamma - 1: the block must be
                                replaced (Sec. 3.1; Algorithm 1, reload branch)           */
    PA_ERR_ARG = -1,         /* bad argument (NULL pointer, r < 1, r >= n, n < 2, ...)  */
    PA_ERR_NO_GAMMA = -2,    /* no known Mersenne exponent exceeds r                    */
    PA_ERR_GAMMA = -3,       /* requested gamma is not a Mersenne exponent or <= r      */
    PA_ERR_INEXACT = -4,     /* limb width B too wide: k*L*(2^B-1)^2 >= p0*p1*p2       */
    PA_ERR_SEED_B_EVEN = -5, /* b is even (MH needs gcd(b, 2) = 1, Sec. 2.2 eq. (3))    */
    PA_ERR_SEED_RANGE = -6,  /* a seed word has a bit >= gamma set                      */
    PA_ERR_NOMEM = -7,       /* device allocation failed                                */
    PA_ERR_DEVICE = -8,      /* a HIP call failed                                       */
    PA_ERR_BUSY = -9,        /* no free slot / queue full                               */
    PA_ERR_LIMIT = -10       /* shape outside the supported range (see pa_plan_create)  */
} pa_status;

/* Plan request.  gamma = 0 picks the smallest Mersenne exponent above r.
 * The product of two L-limb numbers needs a cyclic convolution of length
 * N >= 2L - 1; N is a power of two, three times one or five times one (a
 * radix-3 or radix-5 step over three or five power-of-two transforms;
 * N <= 3 * 2^23 and N <= 5 * 2^20), whichever is cheapest among the exact
 * choices by the library's cost model.
 * B = 0 picks the limb width (at most 32 bits) that gives the cheapest exact
 * transform, the widest among equals; otherwise 8 <= B <= 32.  At most one
 * length flag may be set.  The output never depends on B or N. */
#define PA_FLAG_POW2_LENGTHS 1u   /* flags: power-of-two transform lengths only   */
#define PA_FLAG_RADIX3_LENGTHS 2u /* flags: lengths 3 * 2^m only                  */
#define PA_FLAG_RADIX5_LENGTHS 4u /* flags: lengths 5 * 2^m only (m <= 20)        */
typedef struct pa_params {
    uint64_t n;       /* input key length in bits, n >= 2                    */
    uint64_t r;       /* output length in bits, 1 <= r < n and r < gamma     */
    uint64_t gamma;   /* Mersenne exponent, or 0 for automatic               */
    uint32_t B;       /* limb width in bits (the paper's 2^B-ary words), 0 = auto */
    uint32_t flags;   /* 0 or one of the PA_FLAG_*_LENGTHS                  */
    uint32_t col_lg;  /* columns per tile of the key-chunk column pass,
                         2^col_lg; 0 = automatic; otherwise at most the row
                         length 2^log2N2, with log2N1 + col_lg <= 14       */
    uint32_t reserved; /* must be 0                                          */
} pa_params;

typedef struct pa_plan_info {
    uint64_t n, r, gamma, k;
    uint32_t B;             /* limb width                                   */
    uint32_t log2N;         /* NTT length N = len_factor * 2^log2N >= 2L - 1 */
    uint64_t L;             /* limbs per gamma-bit number, ceil(gamma/B)    */
    uint64_t N;
    uint64_t key_words;     /* ceil(n/64)                                   */
    uint64_t seed_words;    /* W = ceil(gamma/64), words per seed chunk     */
    uint64_t a_words;       /* k * W                                        */
    uint64_t out_words;     /* ceil(r/64)                                   */
    uint64_t workspace_bytes; /* device memory owned by the plan            */
    double exact_log2;      /* log2(k * L * (2^B - 1)^2); below log2(p0 p1 p2) */
    uint32_t log2N1;        /* column-pass length 2^log2N1                  */
    uint32_t log2N2;        /* row-pass length 2^log2N2 (2^log2N = 2^(log2N1 + log2N2)) */
    uint32_t nprimes;       /* NTT primes per transform (3)                 */
    uint32_t primes[3];     /* the NTT primes p0, p1, p2 of this length     */
    uint32_t len_factor;    /* 1, 3 or 5 (N = len_factor * 2^log2N)         */
    uint32_t col_lg;        /* column-tile width exponent of the key-chunk pass */
} pa_plan_info;

typedef struct pa_plan pa_plan;

/* Create a plan for one (n, r) shape on HIP device `hip_device`: derives
 * (gamma, k, B, L, N), checks that every convolution coefficient stays below
 * the product of the three NTT primes of length N (the three largest primes
 * below 2^30 with N | p - 1; PA_ERR_INEXACT otherwise), allocates the
 * workspace and builds the twiddle tables.  Supported range: k <= 4096 and
 * N <= 2^24 or N = 3 * 2^m <= 3 * 2^23 (PA_ERR_LIMIT otherwise).  On success
 * *out owns device memory until pa_plan_destroy. */
pa_status pa_plan_create(const pa_params *params, int hip_device, pa_plan **out);

/* Derive the shape pa_plan_create would use, without touching any device:
 * same checks and same return codes, and *info filled on PA_OK (its
 * workspace_bytes is what pa_plan_create would allocate). */
pa_status pa_plan_query(const pa_params *params, pa_plan_info *info);

/* Fill *info with the derived shape of a plan. */
pa_status pa_plan_get_info(const pa_plan *plan, pa_plan_info *info);

/* Free a plan and its device memory.  NULL is ignored. */
void pa_plan_destroy(pa_plan *plan);

/* Hash one block (Algorithm 1) and wait for it: enqueues every kernel on
 * `stream` (NULL = default stream), then synchronises the stream and returns
 * the block's status.  On PA_OK, out holds z. */
pa_status pa_hash(pa_plan *plan, const uint64_t *key, const uint64_t *a, const uint64_t *b,
                  const uint64_t *c, uint64_t *out, hipStream_t stream);

/* Same work as pa_hash but returns as soon as it is enqueued: the block's
 * status flags are written to the device word *d_status (decode them with
 * pa_decode_status after the stream has reached this point).  Returns PA_OK
 * if everything was enqueued, or a host-side error. */
pa_status pa_hash_async(pa_plan *plan, const uint64_t *key, const uint64_t *a,
                        const uint64_t *b, const uint64_t *c, uint64_t *out,
                        uint32_t *d_status, hipStream_t stream);

/* Debug variant of pa_hash that also writes the two stage values: y (the MMH
 * output, W words) and U (the MH value before truncation, W words), both
 * device buffers.  Used to check the stage invariants (linearity of MMH over
 * Z_p, affinity of U in y) without the oracle. */
pa_status pa_hash_stages(pa_plan *plan, const uint64_t *key, const uint64_t *a,
                         const uint64_t *b, const uint64_t *c, uint64_t *out,
                         uint64_t *y_out, uint64_t *U_out, hipStream_t stream);

/* Debug aid (determinism check): enqueue on `stream` a fill of every word of
 * the plan's scratch memory (transform arrays, residues, digit sums, limbs,
 * carry functions, flags: everything the plan owns except the twiddle
 * tables) with `word`.  A hash reads no scratch word that it has not written
 * itself, so its result must not depend on what the scratch held: tests
 * poison it with patterns between hashes and compare outputs bit for bit.
 * Ordered with the plan's hashes on the same stream; calls that overlap a
 * hash of the same plan on another stream race.  Returns PA_ERR_ARG for a
 * null plan, PA_ERR_DEVICE when the launch fails. */
pa_status pa_plan_fill_scratch(pa_plan *plan, uint32_t word, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Hashing without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops or harnesses that
 * forbid hipMalloc).
 *
 * pa_hash_noalloc does the work of pa_hash_async for the shape *params would
 * give pa_plan_create, without a plan: the plan is derived on the host and
 * every device buffer the hash needs beyond the caller's (transform arrays,
 * residues, digit sums, carry functions, flags and the twiddle tables of the
 * transform length) lives in one static device array of
 * PA_NOALLOC_MAX_BYTES bytes per GPU, owned by the library and held until
 * the process ends.  The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine), enqueues every kernel on `stream` (which
 * must belong to `hip_device`; NULL = default stream) and returns; the
 * block's status flags go to the caller's device word *d_status (decode
 * with pa_decode_status once the stream has reached this point).
 *
 * The array keeps the last call's contents: the twiddle tables of the last
 * transform length are reused when the next call on that GPU has the same
 * length (a key in the array says which length they are for, checked on the
 * device), everything else is rewritten by each call.  All calls on one GPU
 * share the array: calls that overlap on one GPU (on different streams
 * without ordering between them, or from several host threads) race and
 * give wrong results; order them.
 *
 * Arguments and layouts as for pa_hash_async (device buffers owned by the
 * caller, valid until the stream has passed the call).  Returns the plan
 * errors of *params (PA_ERR_ARG, PA_ERR_NO_GAMMA, PA_ERR_GAMMA,
 * PA_ERR_INEXACT, PA_ERR_LIMIT), PA_ERR_ARG for a NULL pointer or a device
 * number outside 0..63, PA_ERR_LIMIT when the block's buffers (256 bytes +
 * pa_plan_info.workspace_bytes) exceed PA_NOALLOC_MAX_BYTES (nothing
 * launched), PA_ERR_DEVICE when a HIP call fails, else PA_OK. */
#define PA_NOALLOC_MAX_BYTES (64u << 20)
pa_status pa_hash_noalloc(const pa_params *params, int hip_device, const uint64_t *key, const uint64_t *a,
                          const uint64_t *b, const uint64_t *c, uint64_t *out, uint32_t *d_status,
                          hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched hashing of independent blocks of uneven size.
 *
 * A QKD post-processing pipeline produces reconciled blocks of varying length
 * and compression ratio (Sec. 4 evaluates blocks from 10^6 to 8*10^8 bits and
 * ratios 0.0972 to 0.2957, Table 3).  pa_hash_batched hashes `count` such
 * blocks in one call; each block is hashed exactly as pa_hash would hash it
 * with a plan for its (n, r) (gamma and B by the plan rule, gamma = 0,
 * B = 0).  The blocks run concurrently on the batch plan's worker streams,
 * so blocks too small to fill the GPU alone overlap.
 */
typedef struct pa_block {
    uint64_t n, r;             /* as pa_params.n, pa_params.r                  */
    const uint64_t *key;       /* device, ceil(n/64) words, as for pa_hash     */
    const uint64_t *a, *b, *c; /* device, k*W, W and W words, as for pa_hash   */
    uint64_t *out;             /* device, ceil(r/64) words                     */
} pa_block;

typedef struct pa_batch_plan pa_batch_plan;

/* Create a batch plan on HIP device `hip_device` for calls of at most
 * `max_blocks` blocks with at most `max_total_bits` key bits in total.  The
 * plan keeps the twiddle tables of every transform length it meets and one
 * scratch arena per worker stream, grown to the largest block that worker
 * has run (device memory owned until pa_batch_plan_destroy).  A batch plan
 * is used by one host thread at a time. */
pa_status pa_batch_plan_create(uint32_t max_blocks, uint64_t max_total_bits, int hip_device,
                               pa_batch_plan **out);

/* Waits for the plan's work, then frees it (NULL is a no-op). */
void pa_batch_plan_destroy(pa_batch_plan *plan);

/* Hash blocks[0..count) (host array of descriptors; device buffers as for
 * pa_hash, valid until the call returns).  The work is ordered after earlier
 * work on `stream`; the call returns when every block is done.
 * per_block[i] (host) receives block i's status: a plan error (PA_ERR_ARG,
 * PA_ERR_NO_GAMMA, PA_ERR_INEXACT, PA_ERR_LIMIT) when its (n, r) admits no
 * plan (nothing launched for it), else the device-detected status (PA_OK,
 * PA_RELOAD, PA_ERR_SEED_B_EVEN, PA_ERR_SEED_RANGE); outputs are written only
 * for PA_OK.  Returns PA_ERR_LIMIT (nothing launched) if count > max_blocks
 * or the key bits exceed max_total_bits, PA_ERR_NOMEM / PA_ERR_DEVICE on a
 * failure of the device, else PA_OK. */
pa_status pa_hash_batched(pa_batch_plan *plan, const pa_block *blocks, uint32_t count,
                          pa_status *per_block, hipStream_t stream);

/* Graph replay for repeated batches (enable = 1; 0 turns it off and frees
 * the graphs).  With it on, pa_hash_batched captures the kernel launches of
 * a block list (fork to the worker streams, every block's kernels, join) into
 * a HIP graph the first time it meets that exact list (same descriptors:
 * shapes and buffer addresses) and replays the graph for later calls with
 * the same list, which saves the host-side launch cost of small blocks.  At
 * most 8 lists are kept (least recently used dropped); growing a worker's
 * scratch arena, building tables for a new length or tuning a class
 * (pa_batch_plan_tune) makes the kept graphs stale, and they are captured
 * again when next used.  The results are those of the launches without a
 * graph; the status copy runs outside the graph. */
pa_status pa_batch_plan_set_graphs(pa_batch_plan *plan, int enable);

/* ------------------------------------------------------------------------
 * Autotuning.  The limb width B (the 2^B-ary words of Sec. 2.1), the
 * transform length form (2^m or 3 * 2^m) and the column-tile width change
 * only the speed of a hash, never its output.  The plan rule picks them from
 * a cost model; these calls pick them by timing instead. */

/* Time every candidate shape for *params on HIP device `hip_device` and
 * return the fastest in *best (B, flags and col_lg set explicitly; n, r,
 * gamma copied) and its time per hash in *best_ms (nullable).  Candidates:
 * for each length form admitted by params->flags, the plan rule's limb width
 * for that form and the next narrower exact width that changes the transform
 * length (or params->B alone), each with the rule's column-tile width and its
 * neighbours (or params->col_lg).  Every candidate gets its own plan (those
 * that do not fit in free device memory are skipped) and one warm-up hash;
 * then 5 rounds time `reps` (1..1000) hashes of each candidate in turn, on a
 * private stream, with a random valid key and seeds; a candidate's time is
 * the median of its rounds.  Blocks until done.  Returns the plan errors of
 * *params, PA_ERR_ARG, PA_ERR_NOMEM (no candidate fitted) or PA_ERR_DEVICE. */
pa_status pa_plan_tune(const pa_params *params, int hip_device, uint32_t reps, pa_params *best,
                       double *best_ms);

/* Tune a batch plan for the shapes of blocks[0..count): for each (gamma, k)
 * class not tuned before, pa_plan_tune on the first block of that class
 * (`reps` timed hashes per candidate); later pa_hash_batched calls build
 * every block of a tuned class with the tuned limb width, length form and
 * column-tile width.  Blocks whose (n, r) admits no plan are skipped.  Uses
 * the plan's device; blocks until done; the key and seed buffers of the
 * blocks are not read.  *tuned (nullable) receives the number of classes
 * tuned by this call. */
pa_status pa_batch_plan_tune(pa_batch_plan *plan, const pa_block *blocks, uint32_t count, uint32_t reps,
                             uint32_t *tuned);

/* ------------------------------------------------------------------------
 * Serving: requests from many QKD sessions hashed as they arrive.
 *
 * Each session agrees its random seeds a, b, c (Alg. 1's inputs) once per
 * output class gamma and registers them with pa_server_set_seeds; they stay
 * on the device, and so do their transforms (built on a stream of their own
 * the first time a request of a given transform shape needs them, inside the
 * resident budget, without holding up other requests), so a request costs
 * k + 3 transforms instead of 2k + 4.  A request then carries only its key (host memory in, the
 * r-bit output to host memory out).  pa_submit queues it and returns a
 * ticket at once; a worker thread admits requests in arrival order while one
 * of max_inflight slots is free and the request's device memory (scratch,
 * key, output) fits first-fit into the server's budget, and runs it on the
 * slot's stream (key upload, hash, output download).  pa_poll returns
 * PA_PENDING until the request is done.  A request's result is the same as
 * pa_hash's for the same key and seeds, whatever else is in flight.
 */
typedef struct pa_server_cfg {
    int device;                /* HIP device                                     */
    uint32_t max_inflight;     /* requests running at once, 1..64 (one stream each) */
    uint64_t hbm_budget_bytes; /* device memory for admitted requests (scratch,
                                  key, output), allocated once at creation     */
    uint64_t resident_budget_bytes; /* device memory for the resident sets: the
                                  twiddle tables of each transform length and
                                  the seed transforms of each (session, gamma,
                                  transform shape), allocated once at creation;
                                  sets no admitted request holds are evicted
                                  least recently used first when a new set needs
                                  room; 0: the same as hbm_budget_bytes.  The
                                  registered seeds themselves (8 (kmax + 2) W
                                  bytes each) are outside both budgets        */
} pa_server_cfg;

typedef struct pa_request {
    uint64_t n, r;             /* as pa_params.n, pa_params.r (gamma, B by the plan rule) */
    uint32_t session;          /* seeds registered for (session, gamma)          */
    uint32_t reserved;
    const uint64_t *key;       /* host, ceil(n/64) words; pinned (hipHostMalloc) for
                                  an asynchronous upload; valid until done      */
    uint64_t *out;             /* host, ceil(r/64) words; written when done,
                                  meaningful for PA_OK                           */
} pa_request;

typedef struct pa_timing {
    double queued_ms;          /* submission -> admission (host clock)           */
    double device_ms;          /* key upload start -> output download end (HIP events) */
    double total_ms;           /* submission -> completion seen by the worker    */
} pa_timing;

typedef struct pa_server pa_server;

/* Create a server (allocates the budget, starts the worker thread). */
pa_status pa_server_create(const pa_server_cfg *cfg, pa_server **out);

/* Stop accepting requests, finish the queued and running ones, free
 * everything (NULL is a no-op).  Tickets not yet polled are dropped. */
void pa_server_destroy(pa_server *server);

/* Register the seeds of `session` for output class `gamma` (a tabled Mersenne
 * exponent, PA_ERR_GAMMA otherwise): a = kmax chunks of W = ceil(gamma/64)
 * words (requests of this class need k <= kmax), b and c W words each, host
 * memory, copied before the call returns.  Validity (bits >= gamma clear,
 * b odd) is checked per request on the device, as for pa_hash.  Seeds once
 * registered are not replaced (PA_ERR_BUSY). */
pa_status pa_server_set_seeds(pa_server *server, uint32_t session, uint64_t gamma, uint64_t kmax,
                              const uint64_t *a, const uint64_t *b, const uint64_t *c);

/* Queue a request; *ticket identifies it.  Returns at once: a plan error for
 * (n, r), PA_ERR_ARG when the session has no seeds for the request's gamma
 * (or too few chunks), PA_ERR_LIMIT when the request alone exceeds the
 * budget or its twiddle tables and seed transforms together exceed the
 * resident budget, PA_ERR_BUSY while the server is stopping, else PA_OK.  A
 * queued request is admitted when a slot is free, its memory fits the
 * budget and its resident sets are present or can be placed. */
pa_status pa_submit(pa_server *server, const pa_request *request, uint64_t *ticket);

/* PA_PENDING while the request is queued or running; PA_OK once it is done,
 * with its status in *result (as pa_hash would return it) and, if timing is
 * not NULL, its timing.  A ticket is reported done once; polling it again,
 * or an unknown ticket, gives PA_ERR_ARG. */
pa_status pa_poll(pa_server *server, uint64_t ticket, pa_status *result, pa_timing *timing);

/* Phases of the per-block launch sequence, for pa_plan_read_profile.  Each
 * of the NTT phases is exactly one kernel launch. */
typedef enum pa_phase {
    PA_PH_PROLOGUE = 0,   /* no launch (the seed checks run in the fold); 0   */
    PA_PH_MMH_COL = 1,    /* unpack + forward column pass of 2k arrays, reload check */
    PA_PH_MMH_ROW = 2,    /* row pass: k pairs forward, multiply-accumulate, inverse */
    PA_PH_MMH_COLINV = 3, /* inverse column pass -> convolution coefficients */
    PA_PH_FOLD = 4,       /* Mersenne fold + carry scans -> y                */
    PA_PH_MH_COL = 5,     /* unpack + forward column pass of y and b         */
    PA_PH_MH_ROW = 6,     /* row pass: forward, multiply, inverse            */
    PA_PH_MH_COLINV = 7,  /* inverse column pass                             */
    PA_PH_MH_CARRY = 8,   /* + c, carry scan mod 2^gamma -> U, output z, status */
    PA_PH_FINISH = 9,     /* pa_hash_stages only: y and U packed into words  */
    PA_PH_COUNT = 10
} pa_phase;

/* Per-phase timing.  phase_mask bit p (1u << PA_PH_...) set: every hash call
 * on this plan records a HIP event pair around phase p on the call's stream;
 * 0 turns timing off, PA_PROFILE_ALL times every phase.  Each pair costs a
 * few microseconds of stream time, so a throughput measurement should time
 * only the phase it reports. */
#define PA_PROFILE_ALL ((1u << PA_PH_COUNT) - 1u)
pa_status pa_plan_set_profiling(pa_plan *plan, uint32_t phase_mask);

/* Wait for every recorded event, then return the summed milliseconds and the
 * number of recorded calls per phase since the previous read (arrays of
 * PA_PH_COUNT entries, host memory), and reset the sums. */
pa_status pa_plan_read_profile(pa_plan *plan, double *ms, uint64_t *calls);

/* Measurement utility: the VALU rate the transform kernels' instruction mix
 * reaches on HIP device `hip_device` when nothing else limits it.  Runs two
 * register-only probe kernels on every SIMD (blocking, a few milliseconds):
 * independent lazy radix-2 butterflies modulo a prime below 2^30 (sum
 * reduced to [0, 2p), difference shifted by 2p, Montgomery product: eight
 * VALU instructions, three of them 32x32 -> 64-bit multiply-adds or 32-bit
 * multiplies), and a stream of plain 32-bit adds and xors of the same
 * shape.  *bfly_per_s receives butterflies per second, *plain_per_s lane
 * instructions per second.  Returns PA_ERR_ARG, PA_ERR_NOMEM,
 * PA_ERR_DEVICE or PA_OK. */
pa_status pa_probe_valu(int hip_device, double *bfly_per_s, double *plain_per_s);

/* Measurement utility for the transform design: the rate of lazy radix-2
 * butterflies modulo the 64-bit prime P = 2^64 - 2^32 + 1, whose 2^m-th roots
 * of 2 (m <= 26) a single-prime weighted transform (Crandall-Fagin) of the
 * products mod 2^gamma - 1 would need, on HIP device `hip_device`.  Same
 * register-only setup as pa_probe_valu; *mul_bfly_per_s receives butterflies
 * per second with a general 64-bit twiddle product, *shift_bfly_per_s with
 * twiddles 2^(3j) (those of a 64-point DFT modulo P, 2 having order 192),
 * whose products are shifts.  Returns PA_ERR_ARG, PA_ERR_NOMEM,
 * PA_ERR_DEVICE or PA_OK. */
pa_status pa_probe_goldilocks(int hip_device, double *mul_bfly_per_s, double *shift_bfly_per_s);

/* Map a device status word written by pa_hash_async to a status code. */
pa_status pa_decode_status(uint32_t flags);

/* Static string naming a status code. */
const char *pa_status_string(pa_status status);

#ifdef __cplusplus
}
#endif

#endif /* PA_H */
