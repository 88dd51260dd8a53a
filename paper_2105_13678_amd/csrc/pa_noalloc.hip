// pa_hash_noalloc: the hash of one block without any allocation, for callers
// that cannot allocate device memory.  Every per-call buffer and the twiddle
// tables of the block's transform length live in one static device array per
// GPU, whose device address is looked up once per device.
//
// Layout of the array: [0, 256) a header whose first word is the key of the
// twiddle tables it holds; then the tables of the last transform length
// used; then the per-call scratch of the block (transform arrays, residues,
// digit sums, carry functions, flags).  A call whose length matches the
// header's key reuses the tables (the table kernels see the key on the device
// and return at once), so a captured graph that replays an older length still
// rebuilds what it needs.
#include <mutex>

#include "pa_internal.hpp"

namespace {

constexpr size_t kHeaderBytes = 256;

// The library-owned memory of pa_hash_noalloc on each GPU.  In host code this
// name is not a device address; only the pointer from hipGetSymbolAddress is.
static __device__ __align__(256) uint8_t scratch[PA_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, null until looked up

// Device address of the array on device `dev`, which must be current.
pa_status scratch_of(int dev, char **ptr) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return PA_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *ptr = (char *)g_scratch_ptr[dev];
    return PA_OK;
}

// Key of a twiddle-table set: the tables depend only on the transform length
// (its primes) and its split into column and row lengths.  Never 0, the
// array's initial contents.
uint32_t table_key(const pa_plan &p) { return 0x5A000000u | p.mix << 16 | p.m1 << 8 | p.m2; }

}  // namespace

extern "C" pa_status pa_hash_noalloc(const pa_params *params, int hip_device, const uint64_t *key,
                                     const uint64_t *a, const uint64_t *b, const uint64_t *c, uint64_t *out,
                                     uint32_t *d_status, hipStream_t stream) {
    if (!params || !key || !a || !b || !c || !out || !d_status) return PA_ERR_ARG;
    if (hip_device < 0 || hip_device >= kMaxDevices) return PA_ERR_ARG;
    pa_plan plan{};
    pa::PlanLayout lay;
    pa_status st = pa::derive_plan(params, &plan, &lay);
    if (st != PA_OK) return st;
    if (kHeaderBytes + lay.total > (size_t)PA_NOALLOC_MAX_BYTES) return PA_ERR_LIMIT;
    plan.device = hip_device;
    pa::DeviceGuard guard(hip_device);
    if (!guard.ok) return PA_ERR_DEVICE;
    char *base = nullptr;
    st = scratch_of(hip_device, &base);
    if (st != PA_OK) return st;
    uint32_t *hdr = (uint32_t *)base;
    pa::bind_tables(&plan, base + kHeaderBytes, lay);
    pa::bind_scratch(&plan, base + kHeaderBytes + lay.table_bytes, lay);
    if (pa::launch_twiddles(&plan, stream, hdr, table_key(plan)) != hipSuccess) {
        (void)hipGetLastError();
        return PA_ERR_DEVICE;
    }
    return pa::enqueue_hash(&plan, key, a, b, c, out, d_status, nullptr, nullptr, stream);
}
