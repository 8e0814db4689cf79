// persistent.hip -- one launch advances many chains (or one long chain) by
// many passes. Blocks claim work items in increasing order from a counter:
// resident rings first (each whole run in one item, on chip), then pass by
// pass one item per (chain, cluster). A cluster item of pass e waits until
// its own cluster and both neighbours have finished pass e-1 (progress
// flags), so passes overlap across the chip instead of ending at a kernel
// boundary. Each cluster item is the same cluster pass as the fused kernel
// (Sec. 2.3 overlap carried over several steps) and each resident item the
// same run as the resident kernel, so results are identical bits.
//
// Memory ordering: a finished item's stores are released at agent scope
// before its flag is set; a waiting item acquires at agent scope after it
// sees the flags, so the neighbour data is visible across XCDs. Every wait is
// bounded: past the limit the error word is set and the item goes on, so
// every block always exits.
#include <atomic>

#include "cluster.hpp"

namespace chainrk4 {
namespace {

// A value every lane holds alike, moved to a scalar register.
__device__ __forceinline__ long long uniform64(long long x) {
    const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(x));
    const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(x >> 32));
    return static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo);
}

// The same for a pointer, a double and a chain's state pointers. The chain
// table is read with ordinary loads (the kernel writes global memory, so the
// compiler cannot prove them uniform); moving what every lane holds alike to
// scalar registers keeps it out of the vector registers of the cluster pass.
template <class T>
__device__ __forceinline__ T *uniform_ptr(T *p) {
    return reinterpret_cast<T *>(uniform64(reinterpret_cast<long long>(p)));
}

__device__ __forceinline__ double uniform_f64(double x) {
    return __builtin_bit_cast(double, uniform64(__builtin_bit_cast(long long, x)));
}

__device__ __forceinline__ StateRef uniform_ref(const StateRef &r) {
    return StateRef{uniform_ptr(r.q), uniform_ptr(r.p), uniform_ptr(r.cq), uniform_ptr(r.cp),
                    uniform_ptr(r.z)};
}

// Kept sites [start, start + keep) of cluster g: the wide clusters first,
// then the narrow ones, each class in balanced 4-site units; the last cluster
// also keeps the n % 4 remainder. The host's planner uses the same rule.
__device__ __forceinline__ void cluster_span(const BatchChain &ch, int g, int64_t &start,
                                             int64_t &keep) {
    const int64_t n = uniform64(ch.n), uq = uniform64(ch.uq), ur = uniform64(ch.ur);
    const int G = __builtin_amdgcn_readfirstlane(ch.clusters);
    const int wide = __builtin_amdgcn_readfirstlane(ch.wide);
    int64_t units;
    if (g < wide) {
        start = 4 * (static_cast<int64_t>(g) * uq + (g < ur ? g : ur));
        units = uq + (g < ur ? 1 : 0);
    } else {
        const int h = g - wide;
        const int nuq = __builtin_amdgcn_readfirstlane(ch.nuq);
        const int nur = __builtin_amdgcn_readfirstlane(ch.nur);
        start = 4 * (wide * uq + ur + static_cast<int64_t>(h) * nuq + (h < nur ? h : nur));
        units = nuq + (h < nur ? 1 : 0);
    }
    keep = (g == G - 1) ? n - start : 4 * units;
}

__device__ __forceinline__ int pass_steps(const BatchChain &ch, int e, int depth) {
    if (e < ch.nhead) return e == 0 ? ch.head0 : ch.head1;
    if (ch.tail > 0 && e == ch.passes - 1) return ch.tail;
    return depth;
}

// COH: cluster data moves through device-coherent loads and stores, and the
// hand-off only waits for them to complete. Otherwise: ordinary accesses with
// an agent-scope release (cache write-back) and acquire (invalidate).
// RES: the launch has resident-ring items. Without them the kernel carries no
// resident path, which leaves the cluster pass more registers per wavefront.
// Up to 8 sites per lane without RES the kernel is held to 128 registers (4
// wavefronts per SIMD): the narrow clusters' step loop, which has no LDS
// exchange, would otherwise be scheduled into 132 and cost a wavefront per
// SIMD; held to 128 it keeps one 8-byte spill outside the step loops.
template <int M, class R, bool KAHAN, int S, bool COH, bool RES>
__global__ __launch_bounds__(kBatchThreads)
__attribute__((amdgpu_waves_per_eu((S <= 8 && !RES) ? 4 : 1))) void persistent_kernel(BatchArgs a) {
    constexpr int W = kBatchWaves, WPB = kBatchWaves;
    constexpr int RMAX = kBatchResidentSites;
    constexpr int SPT = RMAX / kBatchThreads;
    constexpr int E = 64 * S * W;
    __shared__ SlotsOf<M, R, W, WPB> slots;
    // Resident rings use `ring`; cluster items give each wavefront a staging
    // area for its device-coherent stores. A workgroup runs one item at a
    // time (a barrier separates them), so the two share one LDS buffer.
    constexpr bool STAGED = COH && (S * sizeof(R)) % 16 == 0;
    constexpr int RING = RES ? 2 * RMAX : 1;
    constexpr int STAGE = STAGED ? WPB * 64 * S : 1;
    __shared__ __align__(16) R lds_buf[RING > STAGE ? RING : STAGE];
    R *const ring = lds_buf;
    R *const stage = lds_buf;
    __shared__ long long claimed;
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    int pass = 0;  // forward scan position in pass_off (uniform over the block)

    for (;;) {
        if (threadIdx.x == 0)
            claimed = static_cast<long long>(atomicAdd(a.counter, 1ull));
        __syncthreads();
        const long long item = uniform64(claimed);
        __syncthreads();
        if (item >= a.total_items) break;

        if constexpr (RES) {
            if (item < a.n_resident) {
                const BatchChain &ch = a.chains[a.n_tiled + item];
                run_resident<M, R, KAHAN, kBatchThreads, SPT>(ch.front, ch.front,
                                                              static_cast<int>(ch.n), ch.nsteps,
                                                              ch.dt, ring);
                continue;
            }
        }

        const int64_t j = item - a.n_resident;
        while (a.pass_off[pass + 1] <= j) ++pass;
        const int64_t w = j - a.pass_off[pass];
        const int32_t *ic = a.item_chain + kBatchWaves * w;
        const int32_t *ig = a.item_cluster + kBatchWaves * w;
        if (__builtin_amdgcn_readfirstlane(ic[1]) == kWideItem) {
            // one wide cluster: the whole workgroup
            const BatchChain &ch = a.chains[__builtin_amdgcn_readfirstlane(ic[0])];
            const int g = __builtin_amdgcn_readfirstlane(ig[0]);
            const int G = ch.clusters;
            int32_t *fl = a.flags + ch.flag_base;
            if (pass > 0) {
                if (threadIdx.x == 0)
                    wait_flags(fl + (g == 0 ? G - 1 : g - 1), fl + g,
                               fl + (g == G - 1 ? 0 : g + 1), pass, a.error, a.spin_limit);
                __syncthreads();
                if constexpr (!COH) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            int64_t start, keep;
            cluster_span(ch, g, start, keep);
            const StateRef in = uniform_ref((pass & 1) ? ch.back : ch.front);
            const StateRef out = uniform_ref((pass & 1) ? ch.front : ch.back);
            const int ksteps = __builtin_amdgcn_readfirstlane(pass_steps(ch, pass, a.depth));
            run_cluster<M, R, KAHAN, S, W, WPB, COH>(in, out, uniform64(ch.n), start - a.halo,
                                                     a.halo, keep, ksteps, uniform_f64(ch.dt),
                                                     &slots, lane, wib, wib, 0,
                                                     STAGED ? stage + wib * 64 * S : nullptr);
            if constexpr (COH)
                drain_memory();
            else
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (threadIdx.x == 0) store_flag(fl + g, pass + 1);
        } else {
            // a pack of narrow clusters: each wavefront runs its own, waits
            // for its own neighbours and marks its own flag
            const int c = __builtin_amdgcn_readfirstlane(ic[wib]);
            if (c != kEmptySlot) {
                const BatchChain &ch = a.chains[c];
                // a slot whose chain has no pass `pass` left is idle
                if (pass < __builtin_amdgcn_readfirstlane(ch.passes)) {
                    const int g = __builtin_amdgcn_readfirstlane(ig[wib]);
                    const int G = ch.clusters;
                    int32_t *fl = a.flags + ch.flag_base;
                    if (pass > 0) {
                        if (lane == 0)
                            wait_flags(fl + (g == 0 ? G - 1 : g - 1), fl + g,
                                       fl + (g == G - 1 ? 0 : g + 1), pass, a.error,
                                       a.spin_limit);
                        // no barrier follows (the wavefront's lanes run
                        // together): keep the compiler from moving the
                        // cluster's loads above the wait
                        if constexpr (COH)
                            __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        else
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    }
                    int64_t start, keep;
                    cluster_span(ch, g, start, keep);
                    const StateRef in = uniform_ref((pass & 1) ? ch.back : ch.front);
                    const StateRef out = uniform_ref((pass & 1) ? ch.front : ch.back);
                    const int ksteps =
                        __builtin_amdgcn_readfirstlane(pass_steps(ch, pass, a.depth));
                    // one wavefront: neighbours by DPP only, no LDS slots
                    run_cluster<M, R, KAHAN, S, 1, WPB, COH>(
                        in, out, uniform64(ch.n), start - a.halo, a.halo, keep, ksteps,
                        uniform_f64(ch.dt), static_cast<SlotsOf<M, R, 1, WPB> *>(nullptr), lane,
                        wib, 0, 0, STAGED ? stage + wib * 64 * S : nullptr);
                    if constexpr (COH)
                        drain_memory();
                    else
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    if (lane == 0) store_flag(fl + g, pass + 1);
                }
            }
        }
        static_assert(E >= 64, "cluster");
    }
}

template <int M, class R, bool KAHAN, int S, bool COH, bool RES>
int capacity_one() {
    static std::atomic<int> cached[64];  // batches on different threads may ask at once
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int v = cached[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu,
                                                         persistent_kernel<M, R, KAHAN, S, COH, RES>,
                                                         kBatchThreads, 0) != hipSuccess)
            return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        v = per_cu * cus;
        cached[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

template <int M, class R, bool KAHAN>
int capacity_s(int s, bool res) {
    switch (s) {
    case 4: return res ? capacity_one<M, R, KAHAN, 4, true, true>()
                       : capacity_one<M, R, KAHAN, 4, true, false>();
    case 8: return res ? capacity_one<M, R, KAHAN, 8, true, true>()
                       : capacity_one<M, R, KAHAN, 8, true, false>();
    case 16: return res ? capacity_one<M, R, KAHAN, 16, true, true>()
                        : capacity_one<M, R, KAHAN, 16, true, false>();
    default: return 0;
    }
}

template <int M, class R, bool KAHAN, bool COH, bool RES>
hipError_t launch_c(int s, int blocks, const BatchArgs &a, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>(blocks)), block(kBatchThreads);
    switch (s) {
    case 4: persistent_kernel<M, R, KAHAN, 4, COH, RES><<<grid, block, 0, st>>>(a); break;
    case 8: persistent_kernel<M, R, KAHAN, 8, COH, RES><<<grid, block, 0, st>>>(a); break;
    case 16: persistent_kernel<M, R, KAHAN, 16, COH, RES><<<grid, block, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int M, class R, bool KAHAN>
hipError_t launch_s(int s, int blocks, const BatchArgs &a, hipStream_t st) {
    const bool res = a.n_resident > 0;
    if (a.fences)
        return res ? launch_c<M, R, KAHAN, false, true>(s, blocks, a, st)
                   : launch_c<M, R, KAHAN, false, false>(s, blocks, a, st);
    return res ? launch_c<M, R, KAHAN, true, true>(s, blocks, a, st)
               : launch_c<M, R, KAHAN, true, false>(s, blocks, a, st);
}

}  // namespace

int persistent_capacity(int model, int prec, int s, bool res) {
    if (model == kQuartic)
        return prec == 0 ? capacity_s<kQuartic, double, false>(s, res)
                         : capacity_s<kQuartic, float, true>(s, res);
    return prec == 0 ? capacity_s<kHarmonic, double, false>(s, res)
                     : capacity_s<kHarmonic, float, true>(s, res);
}

hipError_t launch_persistent(int model, int prec, int s, int blocks, const BatchArgs &a,
                             hipStream_t st) {
    if (blocks < 1) return hipErrorInvalidValue;
    if (model == kQuartic)
        return prec == 0 ? launch_s<kQuartic, double, false>(s, blocks, a, st)
                         : launch_s<kQuartic, float, true>(s, blocks, a, st);
    return prec == 0 ? launch_s<kHarmonic, double, false>(s, blocks, a, st)
                     : launch_s<kHarmonic, float, true>(s, blocks, a, st);
}

}  // namespace chainrk4
