// Register-only probe of the VALU rate for the transform kernels'
// instruction mix, the ceiling their butterfly rate is measured against.
//
// The transform kernels spend their time in lazy radix-2 butterflies modulo
// primes below 2^30 (ntt_device.hpp): a sum reduced to [0, 2p) (add, sub,
// min), a difference shifted by 2p (add, sub) and a Montgomery product
// without final subtraction (v_mad_u64_u32, v_mul_lo_u32, v_mad_u64_u32):
// eight VALU instructions.  Counting every instruction as one issue slot
// (4 cycles per wave64 instruction on a 16-lane SIMD) gives 256 CUs x 64
// lanes x 2.4 GHz / 8 = 4.92 T butterflies/s; the 64-bit multiply-adds may
// occupy the SIMD longer.  The probe runs independent butterflies on
// register-resident values in every lane of every SIMD (no memory traffic,
// no LDS, full occupancy) and reports the rate it reaches, next to the rate
// of a stream of plain 32-bit adds and xors of the same shape.
#include <hip/hip_runtime.h>

#include "ntt_device.hpp"
#include "pa_internal.hpp"

namespace {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_PAIRS = 8;  // independent butterflies per round and thread

// PROBE_PAIRS butterflies per round on pairs (j, j + PROBE_PAIRS), values in
// [0, 2p) throughout; the result is stored so that nothing is dropped.
__global__ __launch_bounds__(PROBE_THREADS) void k_probe_bfly(uint32_t *out, uint32_t rounds, pa::PrimeConst M) {
    uint32_t v[2 * PROBE_PAIRS];
#pragma unroll
    for (int j = 0; j < 2 * PROBE_PAIRS; ++j) v[j] = (threadIdx.x * 2 * PROBE_PAIRS + j + 1) % M.p;
    const uint32_t w = M.w16[1];
    for (uint32_t r = 0; r < rounds; ++r) {
#pragma unroll
        for (int j = 0; j < PROBE_PAIRS; ++j) {
            const uint32_t u = v[j], x = v[j + PROBE_PAIRS];
            v[j] = pa::red2(u + x, M);
            v[j + PROBE_PAIRS] = pa::mont(u + M.p2 - x, w, M);
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < 2 * PROBE_PAIRS; ++j) acc ^= v[j];
    out[blockIdx.x * PROBE_THREADS + threadIdx.x] = acc;
}

// The same loop shape with two plain 32-bit instructions per pair.
__global__ __launch_bounds__(PROBE_THREADS) void k_probe_plain(uint32_t *out, uint32_t rounds, uint32_t seed) {
    uint32_t v[2 * PROBE_PAIRS];
#pragma unroll
    for (int j = 0; j < 2 * PROBE_PAIRS; ++j) v[j] = threadIdx.x * 2 * PROBE_PAIRS + j + seed;
    for (uint32_t r = 0; r < rounds; ++r) {
#pragma unroll
        for (int j = 0; j < PROBE_PAIRS; ++j) {
            v[j] = v[j] + v[j + PROBE_PAIRS];
            v[j + PROBE_PAIRS] = v[j + PROBE_PAIRS] ^ v[j];
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < 2 * PROBE_PAIRS; ++j) acc ^= v[j];
    out[blockIdx.x * PROBE_THREADS + threadIdx.x] = acc;
}

// Arithmetic modulo the 64-bit prime P = 2^64 - 2^32 + 1 (2^64 = 2^32 - 1
// mod P), values kept below 2^64 (not necessarily below P): the instruction
// mix a single-prime weighted transform would run instead of three 30-bit
// transforms.  Sum and difference fold their carry or borrow back with
// 2^32 - 1 (twice, as a second carry can follow the first); the product is
// the 128-bit product reduced with 2^96 = -1 and 2^64 = 2^32 - 1.
constexpr uint64_t GL_EPS = 0xffffffffull;

__device__ __forceinline__ uint64_t gl_add(uint64_t a, uint64_t b) {
    uint64_t s = a + b;
    const uint64_t c1 = s < a ? GL_EPS : 0;
    const uint64_t t = s + c1;
    return t + (t < s ? GL_EPS : 0);
}

__device__ __forceinline__ uint64_t gl_sub(uint64_t a, uint64_t b) {
    const uint64_t d = a - b;
    const uint64_t b1 = a < b ? GL_EPS : 0;
    const uint64_t t = d - b1;
    return t - (d < b1 ? GL_EPS : 0);
}

__device__ __forceinline__ uint64_t gl_reduce(uint64_t lo, uint64_t hi) {
    const uint64_t hh = hi >> 32, hl = hi & GL_EPS;
    uint64_t t0 = lo - hh;
    if (lo < hh) t0 -= GL_EPS;  // borrow: 2^64 = 2^32 - 1
    const uint64_t t1 = hl * GL_EPS;
    const uint64_t r = t0 + t1;
    return r + (r < t1 ? GL_EPS : 0);
}

__device__ __forceinline__ uint64_t gl_mul(uint64_t a, uint64_t b) { return gl_reduce(a * b, __umul64hi(a, b)); }

// a * 2^s for 0 < s < 64: the product's two words are shifts
__device__ __forceinline__ uint64_t gl_shl(uint64_t a, int s) { return gl_reduce(a << s, a >> (64 - s)); }

// PROBE_PAIRS butterflies per round modulo P: with a general twiddle (SHIFT
// false) or with twiddles 2^(3 (j + 1)), the twiddles of a 64-point DFT
// (8 = 2^3 is a 64th root of unity modulo P: 2 has order 192).
template <bool SHIFT>
__global__ __launch_bounds__(PROBE_THREADS) void k_probe_gl(uint64_t *out, uint32_t rounds, uint64_t w) {
    uint64_t v[2 * PROBE_PAIRS];
#pragma unroll
    for (int j = 0; j < 2 * PROBE_PAIRS; ++j) v[j] = 0x9e3779b97f4a7c15ull * (threadIdx.x * 2 * PROBE_PAIRS + j + 1);
    for (uint32_t r = 0; r < rounds; ++r) {
#pragma unroll
        for (int j = 0; j < PROBE_PAIRS; ++j) {
            const uint64_t u = v[j], x = v[j + PROBE_PAIRS];
            v[j] = gl_add(u, x);
            v[j + PROBE_PAIRS] = SHIFT ? gl_shl(gl_sub(u, x), 3 * (j + 1)) : gl_mul(gl_sub(u, x), w);
        }
    }
    uint64_t acc = 0;
#pragma unroll
    for (int j = 0; j < 2 * PROBE_PAIRS; ++j) acc ^= v[j];
    out[blockIdx.x * PROBE_THREADS + threadIdx.x] = acc;
}

}  // namespace

extern "C" pa_status pa_probe_goldilocks(int hip_device, double *mul_bfly_per_s, double *shift_bfly_per_s) {
    if (!mul_bfly_per_s || !shift_bfly_per_s) return PA_ERR_ARG;
    pa::DeviceGuard guard(hip_device);
    if (!guard.ok) return PA_ERR_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return PA_ERR_DEVICE;
    const unsigned groups = (unsigned)prop.multiProcessorCount * 16;
    const uint32_t rounds = 2048;
    const uint64_t w = 0x40000000003fffffull;  // any word: the probe times the instruction mix
    uint64_t *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    pa_status st = PA_ERR_DEVICE;
    float ms_m = 0.f, ms_s = 0.f;
    if (hipMalloc((void **)&out, (size_t)groups * PROBE_THREADS * 8) != hipSuccess) {
        (void)hipGetLastError();
        return PA_ERR_NOMEM;
    }
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        hipLaunchKernelGGL(k_probe_gl<false>, dim3(groups), dim3(PROBE_THREADS), 0, nullptr, out, 64u, w);
        hipLaunchKernelGGL(k_probe_gl<true>, dim3(groups), dim3(PROBE_THREADS), 0, nullptr, out, 64u, w);
        bool ok = hipEventRecord(e0, nullptr) == hipSuccess;
        hipLaunchKernelGGL(k_probe_gl<false>, dim3(groups), dim3(PROBE_THREADS), 0, nullptr, out, rounds, w);
        ok = ok && hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms_m, e0, e1) == hipSuccess;
        ok = ok && hipEventRecord(e0, nullptr) == hipSuccess;
        hipLaunchKernelGGL(k_probe_gl<true>, dim3(groups), dim3(PROBE_THREADS), 0, nullptr, out, rounds, w);
        ok = ok && hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms_s, e0, e1) == hipSuccess;
        if (ok && ms_m > 0.f && ms_s > 0.f) {
            const double lanes = (double)groups * PROBE_THREADS * rounds * PROBE_PAIRS;
            *mul_bfly_per_s = lanes / (ms_m * 1e-3);
            *shift_bfly_per_s = lanes / (ms_s * 1e-3);
            st = PA_OK;
        }
    }
    (void)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return st;
}

extern "C" pa_status pa_probe_valu(int hip_device, double *bfly_per_s, double *plain_per_s) {
    if (!bfly_per_s || !plain_per_s) return PA_ERR_ARG;
    pa::DeviceGuard guard(hip_device);
    if (!guard.ok) return PA_ERR_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return PA_ERR_DEVICE;
    // the prime constants of the 2^21-point transforms (the largest prime of their triple)
    pa_plan p{};
    pa::init_prime_constants(&p, pa::PRIME_TRIPLES[1].p);
    const unsigned groups = (unsigned)prop.multiProcessorCount * 16;  // 16 workgroups of 4 waves per CU
    const uint32_t rounds = 4096;
    uint32_t *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    pa_status st = PA_ERR_DEVICE;
    float ms_b = 0.f, ms_p = 0.f;
    if (hipMalloc((void **)&out, (size_t)groups * PROBE_THREADS * 4) != hipSuccess) {
        (void)hipGetLastError();
        return PA_ERR_NOMEM;
    }
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        hipLaunchKernelGGL(k_probe_bfly, dim3(groups), dim3(PROBE_THREADS), 0, nullptr, out, 64u, p.primes.c[0]);
        hipLaunchKernelGGL(k_probe_plain, dim3(groups), dim3(PROBE_THREADS), 0, nullptr, out, 64u, 1u);
        bool ok = hipEventRecord(e0, nullptr) == hipSuccess;
        hipLaunchKernelGGL(k_probe_bfly, dim3(groups), dim3(PROBE_THREADS), 0, nullptr, out, rounds, p.primes.c[0]);
        ok = ok && hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms_b, e0, e1) == hipSuccess;
        ok = ok && hipEventRecord(e0, nullptr) == hipSuccess;
        hipLaunchKernelGGL(k_probe_plain, dim3(groups), dim3(PROBE_THREADS), 0, nullptr, out, rounds, 7u);
        ok = ok && hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms_p, e0, e1) == hipSuccess;
        if (ok && ms_b > 0.f && ms_p > 0.f) {
            const double lanes = (double)groups * PROBE_THREADS * rounds * PROBE_PAIRS;
            *bfly_per_s = lanes / (ms_b * 1e-3);         // butterflies per second
            *plain_per_s = 2.0 * lanes / (ms_p * 1e-3);  // lane instructions per second
            st = PA_OK;
        }
    }
    (void)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return st;
}
