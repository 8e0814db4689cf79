// launch.hpp -- internal interface between the host library and the kernel
// translation units. Each kernel file exposes plain host launchers; nothing
// here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chainrk4 {

// Buffers of one chain's state. FP64: q, p are double*. FP32 with compensated
// update: q, p are float* and cq, cp are the float carries.
struct StateRef {
    void *q, *p;
    float *cq, *cp;
};

// One pass of the fused kernel: every cluster (W wavefronts) owns `tile`
// output sites and recomputes `halo` sites on each side, advancing
// `ksteps` <= halo/4 steps. `waves` counts clusters.
struct FusedPass {
    StateRef in, out;
    int64_t n;
    int64_t tile;
    int64_t halo;
    int64_t waves;
    double dt;
    int ksteps;
};

// Whole-ring resident run: one workgroup holds the chain on chip for nsteps.
struct ResidentRun {
    StateRef in, out;  // out may equal in
    int64_t n;
    double dt;
    int64_t nsteps;
};

// Naive method: one kernel per RK stage over memory.
struct NaiveBufs {
    void *k1q, *k1p, *k2q, *k2p, *k3q, *k3p;  // stage slopes
    void *yaq, *yap, *ybq, *ybp;              // stage arguments (ping-pong)
};

constexpr int kResidentThreads = 256;
constexpr int kResidentMaxSites = 4096;   // 16 sites per thread
constexpr int kFusedThreads = 256;        // 4 one-wavefront clusters per block

hipError_t launch_fused(int model, int prec, int sites_per_lane, int waves_per_cluster,
                        const FusedPass &a, hipStream_t s);
hipError_t launch_resident(int model, int prec, const ResidentRun &a, hipStream_t s);
size_t resident_lds_bytes(int prec, int64_t n);
hipError_t launch_naive_step(int model, int prec, StateRef y, const NaiveBufs &b, int64_t n,
                             double dt, hipStream_t s);

// Energy: per-block FP64 partials, then one fixed-order finishing block.
constexpr int kEnergyThreads = 256;
constexpr int kEnergyMaxBlocks = 1024;
int energy_blocks(int64_t n);
hipError_t launch_energy(int model, int prec, StateRef y, int64_t n, double *partials,
                         double *result, hipStream_t s);

hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t s);

}  // namespace chainrk4
