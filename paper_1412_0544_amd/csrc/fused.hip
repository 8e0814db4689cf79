// fused.hip -- the fused, temporally blocked RK4 kernel and the resident
// whole-ring kernel, one launch per pass or per run.
//
// Fused kernel (the GPU form of the granular scheme of Sec. 2.3): a cluster is
// W wavefronts holding E = 64*S*W consecutive sites, S per lane, in
// registers. The middle `tile` sites are kept; `halo` sites on each side are
// loaded only to be recomputed and discarded. The wrong values that enter at
// the cluster edges move one site per stage in general (Sec. 2.3), but only
// one per two stages here, since dq/dt = p is local: with halo =
// 2*range*ksteps (range 1, or 2 with second-neighbour bonds) they never reach
// the kept sites, so one pass over memory advances the chain by `ksteps`
// steps. Inside a wavefront neighbour values move by DPP lane
// shifts; between the wavefronts of a cluster only the two edge coordinates
// go through LDS, with one barrier per stage. Clusters never talk to each
// other. Input and output are different buffers (ping-pong): clusters
// overlap, and updating in place would race.
//
// Resident kernel: one workgroup keeps a whole ring of up to 4096 sites on
// chip (state in registers, stage arguments in LDS) for any number of steps;
// 1024 threads from 257 sites on, so each SIMD has four wavefronts to switch
// between while a stage waits on LDS and the barrier.
#include "cluster.hpp"

namespace chainrk4 {
namespace {

constexpr int fused_block_threads(int W) { return W == 1 ? kFusedThreads : 64 * W; }

// One block per cluster (four one-wavefront clusters when W = 1); the grid
// covers every cluster of the pass.
template <int M, class R, bool KAHAN, int S, int W, class C>
__global__ __launch_bounds__(fused_block_threads(W)) void fused_kernel(FusedPass a) {
    constexpr int WPB = fused_block_threads(W) / 64;  // wavefronts per block
    constexpr int CPB = WPB / W;                       // clusters per block
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;                  // wavefront in block
    const int wic = wib % W;                           // wavefront in cluster
    const int64_t cluster = static_cast<int64_t>(blockIdx.x) * CPB + wib / W;
    __shared__ SlotsOf<M, R, W, WPB> slots;
    // W > 1: a block is exactly one cluster and the grid has no extra blocks,
    // so every wavefront reaches every barrier. W = 1: no barriers.
    if (cluster >= a.waves) return;
    run_cluster<M, R, KAHAN, S, W, WPB, false, C>(a.in, a.out, a.n, cluster * a.tile - a.halo,
                                                  a.halo, a.tile, a.ksteps, a.dt, &slots, lane,
                                                  wib, wic, a.balance ? a.ksteps : 0);
}

template <int M, class R, bool KAHAN, int T, int SPT>
__global__ __launch_bounds__(T) void resident_kernel(ResidentRun a) {
    extern __shared__ __align__(16) unsigned char smem[];
    run_resident<M, R, KAHAN, T, SPT>(a.in, a.out, static_cast<int>(a.n), a.nsteps, a.dt,
                                      reinterpret_cast<R *>(smem));
}

template <int M, class R, bool KAHAN, int S, int W, class C>
hipError_t fused_launch_one(const FusedPass &a, hipStream_t st) {
    constexpr int T = fused_block_threads(W);
    constexpr int clusters_per_block = T / 64 / W;
    const int64_t blocks64 = (a.waves + clusters_per_block - 1) / clusters_per_block;
    if (blocks64 <= 0 || blocks64 > 0x7fffffff) return hipErrorInvalidValue;
    FusedPass b = a;
    // one-wavefront clusters of FP64 state take issue priority by progress
    // when every cluster of the pass is resident at once (see
    // steps_by_progress): +1 to 5% at N = 2^14..2^21 in an A/B on one box; the
    // FP32 plans measured 1% either way, so they keep the default order
    b.balance = W == 1 && std::is_same<R, double>::value &&
                blocks64 <= resident_blocks<fused_kernel<M, R, KAHAN, S, W, C>>(T);
    fused_kernel<M, R, KAHAN, S, W, C><<<dim3(static_cast<unsigned>(blocks64)), dim3(T), 0, st>>>(b);
    return hipGetLastError();
}

template <int M, class R, bool KAHAN, int S, class C>
hipError_t fused_dispatch_w(int w, const FusedPass &a, hipStream_t st) {
    switch (w) {
    case 1: return fused_launch_one<M, R, KAHAN, S, 1, C>(a, st);
    case 2: return fused_launch_one<M, R, KAHAN, S, 2, C>(a, st);
    case 4: return fused_launch_one<M, R, KAHAN, S, 4, C>(a, st);
    case 8: return fused_launch_one<M, R, KAHAN, S, 8, C>(a, st);
    default: return hipErrorInvalidValue;
    }
}

template <int M, class R, bool KAHAN, class C = float>
hipError_t fused_dispatch_s(int s, int w, const FusedPass &a, hipStream_t st) {
    switch (s) {
    case 2: return fused_dispatch_w<M, R, KAHAN, 2, C>(w, a, st);
    case 4: return fused_dispatch_w<M, R, KAHAN, 4, C>(w, a, st);
    case 6:
        // built for the FP64 nearest-neighbour chains only
        if constexpr (std::is_same<R, double>::value && !KAHAN && (M == kQuartic || M == kHarmonic))
            return fused_dispatch_w<M, R, KAHAN, 6, C>(w, a, st);
        else
            return hipErrorInvalidValue;
    case 8: return fused_dispatch_w<M, R, KAHAN, 8, C>(w, a, st);
    case 16: return fused_dispatch_w<M, R, KAHAN, 16, C>(w, a, st);
    default: return hipErrorInvalidValue;
    }
}

template <int M, class R, bool KAHAN>
hipError_t resident_dispatch(const ResidentRun &a, hipStream_t st) {
    const size_t lds = 2 * static_cast<size_t>(a.n) * sizeof(R);
    const dim3 grid(1);
    if (a.n <= kResidentThreadsSmall) {
        resident_kernel<M, R, KAHAN, kResidentThreadsSmall, 1>
            <<<grid, dim3(kResidentThreadsSmall), lds, st>>>(a);
        return hipGetLastError();
    }
    const int spt = static_cast<int>((a.n + kResidentThreads - 1) / kResidentThreads);
    const dim3 block(kResidentThreads);
    if (spt <= 1) resident_kernel<M, R, KAHAN, kResidentThreads, 1><<<grid, block, lds, st>>>(a);
    else if (spt <= 2) resident_kernel<M, R, KAHAN, kResidentThreads, 2><<<grid, block, lds, st>>>(a);
    else if (spt <= 4) resident_kernel<M, R, KAHAN, kResidentThreads, 4><<<grid, block, lds, st>>>(a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

template <int M>
hipError_t fused_dispatch_prec(int prec, int s, int w, const FusedPass &a, hipStream_t st) {
    switch (prec) {
    case 0: return fused_dispatch_s<M, double, false>(s, w, a, st);
    case 1: return fused_dispatch_s<M, float, true>(s, w, a, st);
    case 2: return fused_dispatch_s<M, float, true, double>(s, w, a, st);
    case 3: return fused_dispatch_s<M, float, false>(s, w, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fused(int model, int prec, int s, int w, const FusedPass &a, hipStream_t st) {
    switch (model) {
    case kQuartic: return fused_dispatch_prec<kQuartic>(prec, s, w, a, st);
    case kHarmonic: return fused_dispatch_prec<kHarmonic>(prec, s, w, a, st);
    case kQuarticNNN: return fused_dispatch_prec<kQuarticNNN>(prec, s, w, a, st);
    case kHarmonicNNN: return fused_dispatch_prec<kHarmonicNNN>(prec, s, w, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_resident(int model, int prec, const ResidentRun &a, hipStream_t st) {
    if (a.n < 1 || a.n > kResidentMaxSites) return hipErrorInvalidValue;
    if (model == kQuartic) {
        return prec == 0 ? resident_dispatch<kQuartic, double, false>(a, st)
                         : resident_dispatch<kQuartic, float, true>(a, st);
    }
    return prec == 0 ? resident_dispatch<kHarmonic, double, false>(a, st)
                     : resident_dispatch<kHarmonic, float, true>(a, st);
}

}  // namespace chainrk4
