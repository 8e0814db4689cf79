// noalloc.hip -- the energy of a state held in caller buffers, with no handle
// and no workspace, for callers that cannot allocate device memory.
//
// The energy kernels need per-block partial sums and a result word. Here
// they live in `scratch`, a file-scope device array that the library holds
// for the life of the process (each GPU has its own copy at its own address).
// Host code never passes the array's name to a kernel or a copy: the name is
// a host-side stand-in, not a device address. The first call on a device
// looks up that device's address once and keeps it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "chain_rk4.h"
#include "handle.hpp"
#include "launch.hpp"

using namespace chainrk4;

namespace {

// Partial sums of the energy's first kernel (at most kEnergyMaxBlocks blocks
// for any chain length), then the result on a 256-byte line of its own.
constexpr int kScratchResult = kEnergyMaxBlocks;
constexpr int kScratchDoubles = kEnergyMaxBlocks + 256 / sizeof(double);
// Longest chain the call takes (the library's limit on chain length).
constexpr int64_t kNoAllocMaxSites = int64_t(1) << 40;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's `scratch` (looked up once per device, with
// that device current).
int scratch_address(int dev, double **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        double *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(reinterpret_cast<void **>(&ptr), HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(CHAIN_EHIP, "hipGetSymbolAddress(scratch) gave NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CHAIN_OK;
}

bool energy_model(int32_t m) {
    return m == CHAIN_QUARTIC || m == CHAIN_HARMONIC || m == CHAIN_QUARTIC_NNN ||
           m == CHAIN_HARMONIC_NNN;
}

}  // namespace

extern "C" int chain_rk4_energy_noalloc(int32_t model, int32_t prec, int64_t n, const void *q,
                                        const void *p, const void *cq, const void *cp,
                                        void *stream, double *e_out) {
    if (!e_out) return fail(CHAIN_EINVAL, "e_out is NULL");
    if (!energy_model(model))
        return fail(CHAIN_EINVAL, "model %d has no energy (quartic, harmonic and their NNN forms)",
                    model);
    if (prec != CHAIN_FP64 && prec != CHAIN_FP32_KAHAN && prec != CHAIN_FP32_KAHAN64 &&
        prec != CHAIN_FP32)
        return fail(CHAIN_EINVAL, "unknown precision %d", prec);
    if (n < 1 || n > kNoAllocMaxSites)
        return fail(CHAIN_EINVAL, "n must be in 1..2^40 (got %lld)", (long long)n);
    if (!q || !p) return fail(CHAIN_EINVAL, "q and p must be device pointers");
    const bool carries = has_carries(prec);
    if (carries && (!cq || !cp))
        return fail(CHAIN_EINVAL, "a compensated FP32 state needs both carries");
    if (!carries && (cq || cp))
        return fail(CHAIN_EINVAL, "carries are given only with a compensated FP32 precision");
    if ((reinterpret_cast<uintptr_t>(q) | reinterpret_cast<uintptr_t>(p) |
         reinterpret_cast<uintptr_t>(cq) | reinterpret_cast<uintptr_t>(cp)) & 15)
        return fail(CHAIN_EINVAL, "state arrays must be 16-byte aligned");

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CHAIN_EDEVICE, "device %d out of range", dev);
    if (!is_gfx950(dev)) return fail(CHAIN_EDEVICE, "device %d is not a gfx950 GPU", dev);
    double *ptr = nullptr;
    int rc = scratch_address(dev, &ptr);
    if (rc != CHAIN_OK) return rc;

    // Every partial the finishing kernel reads is written by the first one,
    // so nothing in the scratch needs clearing between calls.
    const hipStream_t s = static_cast<hipStream_t>(stream);
    StateRef y{const_cast<void *>(q), const_cast<void *>(p), const_cast<void *>(cq),
               const_cast<void *>(cp), nullptr};
    hipError_t e = launch_energy(model, prec, y, n, ptr, ptr + kScratchResult, s);
    if (e != hipSuccess) return hip_fail(e, "energy launch");
    double v = 0.0;
    HIP_TRY(hipMemcpyAsync(&v, ptr + kScratchResult, sizeof v, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *e_out = v;
    if (!std::isfinite(v)) return fail(CHAIN_ENONFINITE, "energy is not finite (%g)", v);
    return CHAIN_OK;
}
