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

}  // namespace

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
