// fused.hip -- the fused, temporally blocked RK4 kernel and the resident
// whole-ring kernel.
//
// Fused kernel (the GPU form of the granular scheme of Sec. 2.3): a cluster is
// W wavefronts holding E = 64*S*W consecutive sites, S per lane, in
// registers. The middle `tile` sites are kept; `halo` sites on each side are
// loaded only to be recomputed and discarded. With halo = 4*ksteps the wrong
// values that enter at the cluster edges (one site per stage, Sec. 2.3) never
// reach the kept sites, so one pass over memory advances the chain by
// `ksteps` steps. Inside a wavefront neighbour values move by DPP lane
// shifts; between the wavefronts of a cluster only the two edge coordinates
// go through LDS, with one barrier per stage. Clusters never talk to each
// other. Input and output are different buffers (ping-pong): clusters
// overlap, and updating in place would race.
//
// Resident kernel: one workgroup keeps a whole ring of up to 4096 sites on
// chip (state in registers, stage arguments in LDS) for any number of steps.
#include "launch.hpp"
#include "rk4_device.hpp"

namespace chainrk4 {
namespace {

template <class R, int S>
__device__ __forceinline__ void load_contig(R (&dst)[S], const R *__restrict__ src) {
    if constexpr (sizeof(R) == 8) {
        const double2 *v = reinterpret_cast<const double2 *>(src);
#pragma unroll
        for (int m = 0; m < S / 2; ++m) {
            double2 t = v[m];
            dst[2 * m] = t.x;
            dst[2 * m + 1] = t.y;
        }
    } else {
        const float4 *v = reinterpret_cast<const float4 *>(src);
#pragma unroll
        for (int m = 0; m < S / 4; ++m) {
            float4 t = v[m];
            dst[4 * m] = t.x;
            dst[4 * m + 1] = t.y;
            dst[4 * m + 2] = t.z;
            dst[4 * m + 3] = t.w;
        }
    }
}

template <class R, int S>
__device__ __forceinline__ void store_contig(R *__restrict__ dst, const R (&src)[S]) {
    if constexpr (sizeof(R) == 8) {
        double2 *v = reinterpret_cast<double2 *>(dst);
#pragma unroll
        for (int m = 0; m < S / 2; ++m) v[m] = make_double2(src[2 * m], src[2 * m + 1]);
    } else {
        float4 *v = reinterpret_cast<float4 *>(dst);
#pragma unroll
        for (int m = 0; m < S / 4; ++m)
            v[m] = make_float4(src[4 * m], src[4 * m + 1], src[4 * m + 2], src[4 * m + 3]);
    }
}

// Edge coordinates a wavefront publishes for its neighbours in the cluster,
// double-buffered by stage parity so one barrier per stage suffices.
template <class R, int WPB>
struct EdgeSlots {
    R first[2][WPB];
    R last[2][WPB];
};

// One stage for the S sites of this lane. The right neighbour's first
// coordinate comes in, this lane forms its last bond term, and that term goes
// to the right neighbour lane as its left bond term. At a wavefront edge
// inside the cluster the neighbour coordinate comes from LDS instead, and
// lane 0 forms its left bond term itself (the same operation on the same
// values as the left wavefront's lane 63).
template <int M, int S, int STAGE, int W, int WPB, class R>
__device__ __forceinline__ void lane_stage(R (&Q)[S], R (&P)[S], R (&q)[S], R (&p)[S], R (&aq)[S],
                                           R (&ap)[S], const StepConsts<R> &c,
                                           EdgeSlots<R, WPB> *slots, int lane, int wib, int wic,
                                           int parity) {
    const R first = (STAGE == 1) ? q[0] : Q[0];
    const R last = (STAGE == 1) ? q[S - 1] : Q[S - 1];
    R right = from_right(first);
    if constexpr (W > 1) {
        if (lane == 0) slots->first[parity][wib] = first;
        if (lane == 63) slots->last[parity][wib] = last;
        __syncthreads();
        if (lane == 63 && wic + 1 < W) right = slots->first[parity][wib + 1];
    }
    const R brS = ModelOps<M, R>::bond(right - last);
    R bl0 = from_left(brS);
    if constexpr (W > 1) {
        if (lane == 0 && wic > 0) bl0 = ModelOps<M, R>::bond(first - slots->last[parity][wib - 1]);
    }
    stage_sites<M, S, STAGE>(Q, P, q, p, aq, ap, bl0, brS, c);
}

constexpr int fused_block_threads(int W) { return W == 1 ? kFusedThreads : 64 * W; }

// Registers of one cluster's state (this lane's S sites).
template <class R, bool KAHAN, int S>
struct LaneState {
    R q[S], p[S];
    float cq[KAHAN ? S : 1], cp[KAHAN ? S : 1];
};

// Load this lane's S sites of the cluster starting at unwrapped site e0.
template <class R, bool KAHAN, int S, int E>
__device__ __forceinline__ void load_lane(LaneState<R, KAHAN, S> &st, const FusedPass &a, int64_t e0,
                                          int lo) {
    const int64_t n = a.n;
    const int64_t s0 = e0 + lo;
    const R *qin = static_cast<const R *>(a.in.q);
    const R *pin = static_cast<const R *>(a.in.p);
    if (e0 >= 0 && e0 + E <= n) {
        load_contig<R, S>(st.q, qin + s0);
        load_contig<R, S>(st.p, pin + s0);
        if constexpr (KAHAN) {
            load_contig<float, S>(st.cq, a.in.cq + s0);
            load_contig<float, S>(st.cp, a.in.cp + s0);
        }
    } else {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int64_t i = wrap_index(s0 + j, n);
            st.q[j] = qin[i];
            st.p[j] = pin[i];
            if constexpr (KAHAN) {
                st.cq[j] = a.in.cq[i];
                st.cp[j] = a.in.cp[i];
            }
        }
    }
}

// Store the kept sites of this lane.
template <class R, bool KAHAN, int S, int E>
__device__ __forceinline__ void store_lane(const LaneState<R, KAHAN, S> &st, const FusedPass &a,
                                           int64_t e0, int lo) {
    const int64_t n = a.n;
    const int64_t s0 = e0 + lo;
    R *qout = static_cast<R *>(a.out.q);
    R *pout = static_cast<R *>(a.out.p);
    const int64_t keep_end = E - a.halo;
    if (lo >= a.halo && lo + S <= keep_end && s0 + S <= n) {
        store_contig<R, S>(qout + s0, st.q);
        store_contig<R, S>(pout + s0, st.p);
        if constexpr (KAHAN) {
            store_contig<float, S>(a.out.cq + s0, st.cq);
            store_contig<float, S>(a.out.cp + s0, st.cp);
        }
    } else {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int local = lo + j;
            const int64_t g = s0 + j;
            if (local >= a.halo && local < keep_end && g < n) {
                qout[g] = st.q[j];
                pout[g] = st.p[j];
                if constexpr (KAHAN) {
                    a.out.cq[g] = st.cq[j];
                    a.out.cp[g] = st.cp[j];
                }
            }
        }
    }
}

// Whether a lane prefetches the next cluster's sites into registers: only
// where the extra 4*S registers still leave room for three wavefronts per
// SIMD (state, stage arguments and accumulators take 6 values per site).
template <class R, int S>
constexpr bool fused_prefetch() {
    return S * 6 * static_cast<int>(sizeof(R) / 4) + S * 4 <= 128;
}

// The grid is sized to what the device holds at once; each cluster slot
// walks over clusters with a stride of the whole grid. Where registers allow,
// it loads the next cluster's sites while it computes the current one, so
// memory traffic and arithmetic overlap instead of alternating.
template <int M, class R, bool KAHAN, int S, int W>
__global__ __launch_bounds__(fused_block_threads(W)) void fused_kernel(
    FusedPass a) {
    constexpr int WPB = fused_block_threads(W) / 64;  // wavefronts per block
    constexpr int CPB = WPB / W;                       // clusters per block
    constexpr int E = 64 * S * W;                      // sites per cluster
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;                  // wavefront in block
    const int wic = wib % W;                           // wavefront in cluster
    const int lo = (wic * 64 + lane) * S;              // first site in the cluster
    const int64_t stride = static_cast<int64_t>(gridDim.x) * CPB;
    int64_t cluster = static_cast<int64_t>(blockIdx.x) * CPB + wib / W;
    __shared__ EdgeSlots<R, WPB> slots;
    // With W > 1 a block is one cluster slot, so its wavefronts run the same
    // number of iterations and all reach every barrier.

    constexpr bool PF = fused_prefetch<R, S>();
    LaneState<R, KAHAN, S> cur, nxt;
    if (PF && cluster < a.waves) load_lane<R, KAHAN, S, E>(cur, a, cluster * a.tile - a.halo, lo);
    const StepConsts<R> c(a.dt);
    for (; cluster < a.waves; cluster += stride) {
        const int64_t e0 = cluster * a.tile - a.halo;
        if constexpr (PF) {
            if (cluster + stride < a.waves)
                load_lane<R, KAHAN, S, E>(nxt, a, (cluster + stride) * a.tile - a.halo, lo);
        } else {
            load_lane<R, KAHAN, S, E>(cur, a, e0, lo);
        }
        R Q[S], P[S], aq[S], ap[S];
        for (int st = 0; st < a.ksteps; ++st) {
            lane_stage<M, S, 1, W, WPB>(Q, P, cur.q, cur.p, aq, ap, c, &slots, lane, wib, wic, 0);
            lane_stage<M, S, 2, W, WPB>(Q, P, cur.q, cur.p, aq, ap, c, &slots, lane, wib, wic, 1);
            lane_stage<M, S, 3, W, WPB>(Q, P, cur.q, cur.p, aq, ap, c, &slots, lane, wib, wic, 0);
            lane_stage<M, S, 4, W, WPB>(Q, P, cur.q, cur.p, aq, ap, c, &slots, lane, wib, wic, 1);
            if constexpr (KAHAN)
                final_update_kahan<S>(cur.q, cur.p, cur.cq, cur.cp, aq, ap, c);
            else
                final_update<S>(cur.q, cur.p, aq, ap, c);
        }
        store_lane<R, KAHAN, S, E>(cur, a, e0, lo);
        if constexpr (PF) cur = nxt;
    }
}

// ---------------------------------------------------------------------------
// Resident whole-ring kernel. Thread t owns sites t + 256*j, j < SPT. The
// stage argument Q of every site is published in LDS (two buffers used in
// turn, one barrier per stage); P, the accumulators and the state stay in
// registers.
// ---------------------------------------------------------------------------
template <int M, class R, bool KAHAN, int SPT>
__global__ __launch_bounds__(kResidentThreads) void resident_kernel(ResidentRun a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = static_cast<int>(a.n);
    R *buf0 = reinterpret_cast<R *>(smem);
    R *buf1 = buf0 + n;
    const int t = threadIdx.x;
    const R *qin = static_cast<const R *>(a.in.q);
    const R *pin = static_cast<const R *>(a.in.p);

    R q[SPT], p[SPT], P[SPT], aq[SPT], ap[SPT];
    float cq[SPT], cp[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int i = t + kResidentThreads * j;
        if (i < n) {
            q[j] = qin[i];
            p[j] = pin[i];
            if constexpr (KAHAN) {
                cq[j] = a.in.cq[i];
                cp[j] = a.in.cp[i];
            }
            buf0[i] = q[j];
        }
    }
    __syncthreads();

    const StepConsts<R> c(a.dt);
    for (int64_t st = 0; st < a.nsteps; ++st) {
        // stage j reads its argument from `cur` and publishes the next one
        // (after stage 4: the new coordinates) in `nxt`
#pragma unroll
        for (int stage = 1; stage <= 4; ++stage) {
            const R *cur = (stage & 1) ? buf0 : buf1;
            R *nxt = (stage & 1) ? buf1 : buf0;
#pragma unroll
            for (int j = 0; j < SPT; ++j) {
                const int i = t + kResidentThreads * j;
                if (i < n) {
                    const int im = (i == 0) ? n - 1 : i - 1;
                    const int ip = (i == n - 1) ? 0 : i + 1;
                    const R Qm = cur[im], Qj = cur[i], Qp = cur[ip];
                    R Qn = Qj, Pn = P[j];
                    if (stage == 1) {
                        stage_one<M, 1, R>(Qm, Qj, Qp, p[j], q[j], p[j], aq[j], ap[j], Qn, Pn, c);
                    } else if (stage == 2) {
                        stage_one<M, 2, R>(Qm, Qj, Qp, P[j], q[j], p[j], aq[j], ap[j], Qn, Pn, c);
                    } else if (stage == 3) {
                        stage_one<M, 3, R>(Qm, Qj, Qp, P[j], q[j], p[j], aq[j], ap[j], Qn, Pn, c);
                    } else {
                        stage_one<M, 4, R>(Qm, Qj, Qp, P[j], q[j], p[j], aq[j], ap[j], Qn, Pn, c);
                        if constexpr (KAHAN) {
                            kahan_add(q[j], cq[j], c.h6 * aq[j]);
                            kahan_add(p[j], cp[j], c.h6 * ap[j]);
                        } else {
                            q[j] = fma_r(c.h6, aq[j], q[j]);
                            p[j] = fma_r(c.h6, ap[j], p[j]);
                        }
                        Qn = q[j];  // the next step's first argument
                    }
                    nxt[i] = Qn;
                    if (stage != 4) P[j] = Pn;
                }
            }
            __syncthreads();
        }
    }

    R *qout = static_cast<R *>(a.out.q);
    R *pout = static_cast<R *>(a.out.p);
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int i = t + kResidentThreads * j;
        if (i < n) {
            qout[i] = q[j];
            pout[i] = p[j];
            if constexpr (KAHAN) {
                a.out.cq[i] = cq[j];
                a.out.cp[i] = cp[j];
            }
        }
    }
}

// Blocks the device holds at once for one kernel instance (per device).
template <class K>
int resident_blocks(K kernel, int threads) {
    static int cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
            return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev] = per_cu * cus > 0 ? per_cu * cus : 1;
    }
    return cached[dev];
}

template <int M, class R, bool KAHAN, int S, int W>
hipError_t fused_launch_one(const FusedPass &a, hipStream_t st) {
    constexpr int T = fused_block_threads(W);
    constexpr int clusters_per_block = T / 64 / W;
    int64_t blocks64 = (a.waves + clusters_per_block - 1) / clusters_per_block;
    const int cap = resident_blocks(fused_kernel<M, R, KAHAN, S, W>, T);
    if (cap <= 0) return hipErrorInvalidValue;
    if (blocks64 > cap) blocks64 = cap;
    if (blocks64 <= 0) return hipErrorInvalidValue;
    fused_kernel<M, R, KAHAN, S, W><<<dim3(static_cast<unsigned>(blocks64)), dim3(T), 0, st>>>(a);
    return hipGetLastError();
}

template <int M, class R, bool KAHAN, int S>
hipError_t fused_dispatch_w(int w, const FusedPass &a, hipStream_t st) {
    switch (w) {
    case 1: return fused_launch_one<M, R, KAHAN, S, 1>(a, st);
    case 2: return fused_launch_one<M, R, KAHAN, S, 2>(a, st);
    case 4: return fused_launch_one<M, R, KAHAN, S, 4>(a, st);
    case 8: return fused_launch_one<M, R, KAHAN, S, 8>(a, st);
    default: return hipErrorInvalidValue;
    }
}

template <int M, class R, bool KAHAN>
hipError_t fused_dispatch_s(int s, int w, const FusedPass &a, hipStream_t st) {
    switch (s) {
    case 4: return fused_dispatch_w<M, R, KAHAN, 4>(w, a, st);
    case 8: return fused_dispatch_w<M, R, KAHAN, 8>(w, a, st);
    case 16: return fused_dispatch_w<M, R, KAHAN, 16>(w, a, st);
    default: return hipErrorInvalidValue;
    }
}

template <int M, class R, bool KAHAN>
hipError_t resident_dispatch(const ResidentRun &a, hipStream_t st) {
    const int spt = static_cast<int>((a.n + kResidentThreads - 1) / kResidentThreads);
    const size_t lds = 2 * static_cast<size_t>(a.n) * sizeof(R);
    const dim3 grid(1), block(kResidentThreads);
    if (spt <= 1) resident_kernel<M, R, KAHAN, 1><<<grid, block, lds, st>>>(a);
    else if (spt <= 2) resident_kernel<M, R, KAHAN, 2><<<grid, block, lds, st>>>(a);
    else if (spt <= 4) resident_kernel<M, R, KAHAN, 4><<<grid, block, lds, st>>>(a);
    else if (spt <= 8) resident_kernel<M, R, KAHAN, 8><<<grid, block, lds, st>>>(a);
    else if (spt <= 16) resident_kernel<M, R, KAHAN, 16><<<grid, block, lds, st>>>(a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fused(int model, int prec, int s, int w, const FusedPass &a, hipStream_t st) {
    if (model == kQuartic) {
        return prec == 0 ? fused_dispatch_s<kQuartic, double, false>(s, w, a, st)
                         : fused_dispatch_s<kQuartic, float, true>(s, w, a, st);
    }
    return prec == 0 ? fused_dispatch_s<kHarmonic, double, false>(s, w, a, st)
                     : fused_dispatch_s<kHarmonic, float, true>(s, w, a, st);
}

size_t resident_lds_bytes(int prec, int64_t n) {
    return 2 * static_cast<size_t>(n) * (prec == 0 ? sizeof(double) : sizeof(float));
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
