// cluster.hpp -- device code shared by the fused, resident and persistent
// kernels: one cluster pass (Sec. 2.3 with the overlap carried over several
// steps) and one whole-ring resident run. Every kernel that advances a chain
// goes through these two functions, so every launch shape gives the same bits.
#pragma once

#include <atomic>
#include <type_traits>

#include "launch.hpp"
#include "rk4_device.hpp"

namespace chainrk4 {

// Contiguous loads and stores of a lane's S sites with the widest vector
// access S allows. The address must be aligned to that width: the arrays
// start on 16-byte boundaries, every cluster origin is a whole number of
// 16-byte vectors (the single-chain and batch planners round the halo up to
// one), and a lane's first site is S sites past it.
template <class R, int S>
__device__ __forceinline__ void load_contig(R (&dst)[S], const R *__restrict__ src) {
    if constexpr (sizeof(R) == 8 && S % 2 == 0) {
        const double2 *v = reinterpret_cast<const double2 *>(src);
#pragma unroll
        for (int m = 0; m < S / 2; ++m) {
            double2 t = v[m];
            dst[2 * m] = t.x;
            dst[2 * m + 1] = t.y;
        }
    } else if constexpr (sizeof(R) == 4 && S % 4 == 0) {
        const float4 *v = reinterpret_cast<const float4 *>(src);
#pragma unroll
        for (int m = 0; m < S / 4; ++m) {
            float4 t = v[m];
            dst[4 * m] = t.x;
            dst[4 * m + 1] = t.y;
            dst[4 * m + 2] = t.z;
            dst[4 * m + 3] = t.w;
        }
    } else if constexpr (sizeof(R) == 4 && S % 2 == 0) {
        const float2 *v = reinterpret_cast<const float2 *>(src);
#pragma unroll
        for (int m = 0; m < S / 2; ++m) {
            float2 t = v[m];
            dst[2 * m] = t.x;
            dst[2 * m + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int m = 0; m < S; ++m) dst[m] = src[m];
    }
}

template <class R, int S>
__device__ __forceinline__ void store_contig(R *__restrict__ dst, const R (&src)[S]) {
    if constexpr (sizeof(R) == 8 && S % 2 == 0) {
        double2 *v = reinterpret_cast<double2 *>(dst);
#pragma unroll
        for (int m = 0; m < S / 2; ++m) v[m] = make_double2(src[2 * m], src[2 * m + 1]);
    } else if constexpr (sizeof(R) == 4 && S % 4 == 0) {
        float4 *v = reinterpret_cast<float4 *>(dst);
#pragma unroll
        for (int m = 0; m < S / 4; ++m)
            v[m] = make_float4(src[4 * m], src[4 * m + 1], src[4 * m + 2], src[4 * m + 3]);
    } else if constexpr (sizeof(R) == 4 && S % 2 == 0) {
        float2 *v = reinterpret_cast<float2 *>(dst);
#pragma unroll
        for (int m = 0; m < S / 2; ++m) v[m] = make_float2(src[2 * m], src[2 * m + 1]);
    } else {
#pragma unroll
        for (int m = 0; m < S; ++m) dst[m] = src[m];
    }
}

// Coordinates cross lanes by one of three routes:
//  * one-wavefront cluster: DPP only (the wavefront's edge lanes take values
//    that only reach the halo);
//  * several wavefronts, 8-byte state: DPP inside each wavefront, and the
//    wavefront edge lanes exchange through two LDS slots per wavefront;
//  * several wavefronts, 4-byte state: every lane publishes its edge
//    coordinates in LDS and reads its neighbours' after the stage's barrier
//    (no lane-dependent branches and no DPP moves, which frees registers:
//    the FP32 kernels with 16 sites per lane go from 3 to 4 wavefronts per
//    SIMD; for FP64 state the wider LDS traffic measured slower).
// Every bond term that joins two lanes is formed by the same operation on
// the same two coordinates whichever lane forms it, so the route does not
// change a bit of the result.
template <int W, class R>
constexpr bool all_lane_exchange() {
    return W > 1 && sizeof(R) == 4;
}

// LDS slots, double-buffered by stage parity so one barrier per stage
// suffices. A block of a multi-wavefront cluster holds exactly one cluster.
// ALL: one slot per lane; otherwise one per wavefront.
template <class R, int WPB, bool ALL>
struct EdgeSlots {
    R first[2][ALL ? 64 * WPB : WPB];
    R last[2][ALL ? 64 * WPB : WPB];
};

// The same for next-nearest-neighbour coupling: two coordinates per edge.
template <class R, int WPB, bool ALL>
struct EdgeSlots2 {
    R first[2][ALL ? 64 * WPB : WPB][2];  // [parity][slot][0: Q_0, 1: Q_1]
    R last[2][ALL ? 64 * WPB : WPB][2];   // [parity][slot][0: Q_{S-1}, 1: Q_{S-2}]
};

template <int M, class R, int W, int WPB>
using SlotsOf =
    typename std::conditional<coupling_range<M>() == 2,
                              EdgeSlots2<R, WPB, all_lane_exchange<W, R>()>,
                              EdgeSlots<R, WPB, all_lane_exchange<W, R>()>>::type;

// Lane of the block and its two neighbour lanes in the cluster. The
// outermost lanes of the cluster read their own slot instead (their sites lie
// in the recomputed halo, so any finite value does).
struct LaneNbrs {
    int self, left, right;
};
template <int W, int WPB>
__device__ __forceinline__ LaneNbrs lane_nbrs(int lane, int wib) {
    static_assert(W > 1 && W == WPB, "a block of a multi-wavefront cluster is one cluster");
    constexpr int NL = 64 * W;
    const int t = wib * 64 + lane;
    return {t, t > 0 ? t - 1 : t, t + 1 < NL ? t + 1 : t};
}

// Bond terms that reach past this lane's first and last site, NN coupling:
// bl = bond(first - left neighbour's last), br = bond(right neighbour's
// first - last).
template <int M, int W, int WPB, class R>
__device__ __forceinline__ void edge_bonds(R first, R last, SlotsOf<M, R, W, WPB> *slots, int lane,
                                           int wib, int wic, int parity, R &bl, R &br) {
    using Ops = ModelOps<M, R>;
    if constexpr (all_lane_exchange<W, R>()) {
        const LaneNbrs nb = lane_nbrs<W, WPB>(lane, wib);
        slots->first[parity][nb.self] = first;
        slots->last[parity][nb.self] = last;
        __syncthreads();
        br = Ops::bond(slots->first[parity][nb.right] - last);
        bl = Ops::bond(first - slots->last[parity][nb.left]);
    } else {
        R right = from_right(first);
        if constexpr (W > 1) {
            if (lane == 0) slots->first[parity][wib] = first;
            if (lane == 63) slots->last[parity][wib] = last;
            __syncthreads();
            if (lane == 63 && wic + 1 < W) right = slots->first[parity][wib + 1];
        }
        br = Ops::bond(right - last);
        bl = from_left(br);
        if constexpr (W > 1) {
            if (lane == 0 && wic > 0) bl = Ops::bond(first - slots->last[parity][wib - 1]);
        }
    }
}

// The same with next-nearest-neighbour coupling: three bond terms reach past
// each end (b1: first neighbour; b2a, b2b: the two second-neighbour bonds
// that cross the edge, the outer one first). f0, f1: the lane's first two
// coordinates; l0, l1: its last two, outermost first.
template <int M, int W, int WPB, class R>
__device__ __forceinline__ void edge_bonds2(R f0, R f1, R l0, R l1,
                                            SlotsOf<M, R, W, WPB> *slots, int lane, int wib,
                                            int wic, int parity, R &b1l, R &b2la, R &b2lb,
                                            R &b1r, R &b2ra, R &b2rb) {
    using Ops = ModelOps<M, R>;
    if constexpr (all_lane_exchange<W, R>()) {
        const LaneNbrs nb = lane_nbrs<W, WPB>(lane, wib);
        slots->first[parity][nb.self][0] = f0;
        slots->first[parity][nb.self][1] = f1;
        slots->last[parity][nb.self][0] = l0;
        slots->last[parity][nb.self][1] = l1;
        __syncthreads();
        const R r0 = slots->first[parity][nb.right][0], r1 = slots->first[parity][nb.right][1];
        const R L0 = slots->last[parity][nb.left][0], L1 = slots->last[parity][nb.left][1];
        b1r = Ops::bond(r0 - l0);
        b2ra = Ops::bond(r0 - l1);
        b2rb = Ops::bond(r1 - l0);
        b1l = Ops::bond(f0 - L0);
        b2la = Ops::bond(f0 - L1);
        b2lb = Ops::bond(f1 - L0);
    } else {
        R r0 = from_right(f0), r1 = from_right(f1);
        if constexpr (W > 1) {
            if (lane == 0) {
                slots->first[parity][wib][0] = f0;
                slots->first[parity][wib][1] = f1;
            }
            if (lane == 63) {
                slots->last[parity][wib][0] = l0;
                slots->last[parity][wib][1] = l1;
            }
            __syncthreads();
            if (lane == 63 && wic + 1 < W) {
                r0 = slots->first[parity][wib + 1][0];
                r1 = slots->first[parity][wib + 1][1];
            }
        }
        b1r = Ops::bond(r0 - l0);
        b2ra = Ops::bond(r0 - l1);
        b2rb = Ops::bond(r1 - l0);
        b1l = from_left(b1r);
        b2la = from_left(b2ra);
        b2lb = from_left(b2rb);
        if constexpr (W > 1) {
            if (lane == 0 && wic > 0) {
                const R L0 = slots->last[parity][wib - 1][0];
                const R L1 = slots->last[parity][wib - 1][1];
                b1l = Ops::bond(f0 - L0);
                b2la = Ops::bond(f0 - L1);
                b2lb = Ops::bond(f1 - L0);
            }
        }
    }
}

// One stage for the S sites of this lane.
template <int M, int S, int STAGE, int W, int WPB, class R, bool SPLIT>
__device__ __forceinline__ void lane_stage(R (&Q)[S], R (&X)[S], R (&q)[S], R (&p)[S], R (&s)[S],
                                           R (&a)[S], const StepConsts<R, SPLIT> &c,
                                           SlotsOf<M, R, W, WPB> *slots, int lane, int wib,
                                           int wic, int parity) {
    const R first = (STAGE == 1) ? q[0] : Q[0];
    const R last = (STAGE == 1) ? q[S - 1] : Q[S - 1];
    R bl0, brS;
    edge_bonds<M, W, WPB>(first, last, slots, lane, wib, wic, parity, bl0, brS);
    stage_sites<M, S, STAGE>(Q, X, q, p, s, a, bl0, brS, c);
}

// The same with next-nearest-neighbour coupling.
template <int M, int S, int STAGE, int W, int WPB, class R, bool SPLIT>
__device__ __forceinline__ void lane_stage_nnn(R (&Q)[S], R (&X)[S], R (&q)[S], R (&p)[S],
                                               R (&s)[S], R (&a)[S], const StepConsts<R, SPLIT> &c,
                                               SlotsOf<M, R, W, WPB> *slots, int lane, int wib,
                                               int wic, int parity) {
    const R f0 = (STAGE == 1) ? q[0] : Q[0];
    const R f1 = (STAGE == 1) ? q[1] : Q[1];
    const R l1 = (STAGE == 1) ? q[S - 2] : Q[S - 2];
    const R l0 = (STAGE == 1) ? q[S - 1] : Q[S - 1];
    R b1l0, b2lm2, b2lm1, b1rS, b2rS2, b2rS1;
    edge_bonds2<M, W, WPB>(f0, f1, l0, l1, slots, lane, wib, wic, parity, b1l0, b2lm2, b2lm1,
                           b1rS, b2rS2, b2rS1);
    stage_sites_nnn<M, S, STAGE>(Q, X, q, p, s, a, b1l0, b2lm2, b2lm1, b1rS, b2rS2, b2rS1, c);
}

// Dispatch on the coupling range of the model.
template <int M, int S, int STAGE, int W, int WPB, class R, bool SPLIT>
__device__ __forceinline__ void any_lane_stage(R (&Q)[S], R (&X)[S], R (&q)[S], R (&p)[S],
                                               R (&s)[S], R (&a)[S], const StepConsts<R, SPLIT> &c,
                                               SlotsOf<M, R, W, WPB> *slots, int lane, int wib,
                                               int wic, int parity) {
    if constexpr (coupling_range<M>() == 2)
        lane_stage_nnn<M, S, STAGE, W, WPB>(Q, X, q, p, s, a, c, slots, lane, wib, wic, parity);
    else
        lane_stage<M, S, STAGE, W, WPB>(Q, X, q, p, s, a, c, slots, lane, wib, wic, parity);
}

// Device-coherent element access (memory scope: agent). Stores are written
// through to the point where every XCD sees them and loads are not served
// from a stale cache line, so cluster outputs can be handed to a cluster
// running on another XCD without writing back or invalidating whole caches.
template <class R>
using global_ptr = __attribute__((address_space(1))) R *;

template <class R>
__device__ __forceinline__ R load_coherent(const R *p) {
    return __hip_atomic_load((global_ptr<R>)(const_cast<R *>(p)), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
template <class R>
__device__ __forceinline__ void store_coherent(R *p, R v) {
    __hip_atomic_store((global_ptr<R>)(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-coherent 16-byte stores. The agent-scope relaxed atomics above are
// at most 8 bytes wide, and an 8-byte store each costs a 32-byte memory
// transaction (the batch kernel's stores counted 4x their bytes); a
// buffer store with the device-scope cache policy (sc1, the same policy
// those atomics carry) moves 16 bytes at once. The resource covers one
// cluster's window, so a store can never reach outside it (a buffer access
// beyond the resource is dropped).
constexpr int kRawBufferWord3 = 0x00020000;  // 32-bit data, untyped accesses (gfx9 family)
constexpr int kDeviceCoherent = 16;          // cache policy bit sc1: device scope

__device__ __forceinline__ __amdgpu_buffer_rsrc_t window_rsrc(const void *base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, bytes, kRawBufferWord3);
}

// Store a lane's S values at byte offset `off` of the window, 16 bytes at a time.
template <class R, int S>
__device__ __forceinline__ void store_window(__amdgpu_buffer_rsrc_t r, int off, const R (&src)[S]) {
    static_assert((S * sizeof(R)) % 16 == 0, "whole 16-byte vectors");
    constexpr int P = 16 / sizeof(R);
    using U4 = __attribute__((ext_vector_type(4))) unsigned;
#pragma unroll
    for (int m = 0; m < S / P; ++m) {
        U4 v;
        if constexpr (P == 2)
            v = __builtin_bit_cast(U4, make_double2(src[2 * m], src[2 * m + 1]));
        else
            v = __builtin_bit_cast(U4, make_float4(src[4 * m], src[4 * m + 1], src[4 * m + 2],
                                                   src[4 * m + 3]));
        __builtin_amdgcn_raw_buffer_store_b128(v, r, off + 16 * m, 0, kDeviceCoherent);
    }
}

// Progress flags of clusters handing data to each other inside one launch.
__device__ __forceinline__ int load_flag(const int32_t *f) {
    return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_flag(int32_t *f, int v) {
    __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0: wait until flags f0, f1, f2 reach `need`. Bounded: past
// `spin_limit` polls, or once another wait has given up, the error word is
// set and the caller goes on (its results are then invalid), so every
// workgroup always finishes.
__device__ inline bool wait_flags(const int32_t *f0, const int32_t *f1, const int32_t *f2,
                                  int need, int32_t *error, int spin_limit) {
    for (int spin = 0;; ++spin) {
        if (load_flag(f0) >= need && load_flag(f1) >= need && load_flag(f2) >= need) return true;
        if (spin >= spin_limit || load_flag(error) != 0) {
            store_flag(error, 1);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// Steps with issue priority from progress. A SIMD issues from its oldest
// wavefront first, so when all of a launch's clusters are resident at once
// (one round), the youngest wavefronts lag and end their pass alone, at a
// fraction of the SIMD's rate, while the others have already left. A
// wavefront that lowers its priority as it advances (four levels over
// `total` steps) lets the lagging ones catch up, so those of a SIMD finish
// together. It changes only the order of issue, never a result.
//
// Runs body() for the steps done, ..., done + k - 1 of `total`, setting the
// priority once per run of steps at one level: a branch inside the step loop
// would split its body and cost registers. total = 0 keeps one level.
__device__ __forceinline__ void set_priority_level(int q) {
    switch (q) {
    case 0: __builtin_amdgcn_s_setprio(3); break;
    case 1: __builtin_amdgcn_s_setprio(2); break;
    case 2: __builtin_amdgcn_s_setprio(1); break;
    default: __builtin_amdgcn_s_setprio(0); break;
    }
}

template <class F>
__device__ __forceinline__ void steps_by_progress(int64_t done, int64_t k, int64_t total,
                                                  F &&body) {
    // the three level boundaries, relative to `done`, as 32-bit counts
    int b[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        int64_t x = ((j + 1) * total + 3) / 4 - done;
        b[j] = static_cast<int>(x < 0 ? 0 : (x > k ? k : x));
    }
    const int kk = static_cast<int>(k);
    int t = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int end = q < 3 ? b[q] : kk;
        if (t < end) {
            set_priority_level(q);
            for (; t < end; ++t) body();
        }
    }
}

// Wait until every memory operation this wavefront issued has completed.
__device__ __forceinline__ void drain_memory() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Registers of one lane's S sites.
template <class R, bool KAHAN, int S, class C = float>
struct LaneState {
    R q[S], p[S];
    C cq[KAHAN ? S : 1], cp[KAHAN ? S : 1];   // carries of the compensated update
};

// Whether the device-coherent accesses of a lane's S sites can go 16 bytes
// at a time (state and carries in whole 16-byte vectors).
template <class R, bool KAHAN, int S, class C>
constexpr bool coherent_vectors() {
    return (S * sizeof(R)) % 16 == 0 && (!KAHAN || (S * sizeof(C)) % 16 == 0);
}

// Load this lane's S sites, starting at unwrapped site s0 of a ring of n
// sites. `contiguous` (uniform over the cluster) says the cluster's sites
// need no wrap, so vector loads apply. The device-coherent form (COH) loads
// 8 bytes at a time: 16-byte loads would need their four destination
// registers adjacent, which the state carried through the step loop then
// keeps (that cost the 8-site FP64 batch kernel 16 registers), and the loads'
// neighbouring sectors are served from L2 anyway.
template <class R, bool KAHAN, int S, bool COH = false, class C = float>
__device__ __forceinline__ void load_lane(LaneState<R, KAHAN, S, C> &st, const StateRef &in,
                                          int64_t n, int64_t s0, bool contiguous) {
    const R *qin = static_cast<const R *>(in.q);
    const R *pin = static_cast<const R *>(in.p);
    const C *cqin = static_cast<const C *>(in.cq);
    const C *cpin = static_cast<const C *>(in.cp);
    if constexpr (COH) {
        if (contiguous) {
            const R *qb = qin + s0, *pb = pin + s0;
#pragma unroll
            for (int j = 0; j < S; ++j) {
                st.q[j] = load_coherent(qb + j);
                st.p[j] = load_coherent(pb + j);
                if constexpr (KAHAN) {
                    st.cq[j] = load_coherent(cqin + s0 + j);
                    st.cp[j] = load_coherent(cpin + s0 + j);
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const int64_t i = wrap_index(s0 + j, n);
                st.q[j] = load_coherent(qin + i);
                st.p[j] = load_coherent(pin + i);
                if constexpr (KAHAN) {
                    st.cq[j] = load_coherent(cqin + i);
                    st.cp[j] = load_coherent(cpin + i);
                }
            }
        }
    } else if (contiguous) {
        load_contig<R, S>(st.q, qin + s0);
        load_contig<R, S>(st.p, pin + s0);
        if constexpr (KAHAN) {
            load_contig<C, S>(st.cq, cqin + s0);
            load_contig<C, S>(st.cp, cpin + s0);
        }
    } else {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int64_t i = wrap_index(s0 + j, n);
            st.q[j] = qin[i];
            st.p[j] = pin[i];
            if constexpr (KAHAN) {
                st.cq[j] = cqin[i];
                st.cp[j] = cpin[i];
            }
        }
    }
}

// Store the kept sites of this lane: cluster-local positions
// [keep_lo, keep_hi) that are also below n (lo is the lane's first local
// position, s0 its unwrapped site; kept sites never wrap).
template <class R, bool KAHAN, int S, bool COH = false, class C = float>
__device__ __forceinline__ void store_lane(const LaneState<R, KAHAN, S, C> &st, const StateRef &out,
                                           int64_t n, int64_t s0, int lo, int64_t keep_lo,
                                           int64_t keep_hi, int window = 0) {
    R *qout = static_cast<R *>(out.q);
    R *pout = static_cast<R *>(out.p);
    C *cqout = static_cast<C *>(out.cq);
    C *cpout = static_cast<C *>(out.cp);
    // The lane's sites j in [j0, j1) are kept. Two 32-bit bounds, so that
    // whatever the compiler precomputes of this test before the step loop
    // holds two registers, not a 64-bit bound per site.
    const int j0 = static_cast<int>(keep_lo - lo < 0 ? 0 : (keep_lo - lo > S ? S : keep_lo - lo));
    const int64_t end = (keep_hi - lo < n - s0) ? keep_hi - lo : n - s0;
    const int j1 = static_cast<int>(end < 0 ? 0 : (end > S ? S : end));
    if constexpr (COH && coherent_vectors<R, KAHAN, S, C>()) {
        // kept sites never wrap: the window from the cluster origin s0 - lo
        // is contiguous up to every kept site
        if (j0 == 0 && j1 == S) {
            // the resource spans the cluster's window from its origin (which
            // may lie before the array: only kept sites, inside it, are written)
            const int64_t e0 = s0 - lo;
            store_window<R, S>(window_rsrc(qout + e0, window * sizeof(R)), lo * sizeof(R), st.q);
            store_window<R, S>(window_rsrc(pout + e0, window * sizeof(R)), lo * sizeof(R), st.p);
            if constexpr (KAHAN) {
                store_window<C, S>(window_rsrc(cqout + e0, window * sizeof(C)), lo * sizeof(C),
                                   st.cq);
                store_window<C, S>(window_rsrc(cpout + e0, window * sizeof(C)), lo * sizeof(C),
                                   st.cp);
            }
            return;
        }
    }
    if constexpr (COH) {
        R *qb = qout + s0, *pb = pout + s0;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (j >= j0 && j < j1) {
                store_coherent(qb + j, st.q[j]);
                store_coherent(pb + j, st.p[j]);
                if constexpr (KAHAN) {
                    store_coherent(cqout + s0 + j, st.cq[j]);
                    store_coherent(cpout + s0 + j, st.cp[j]);
                }
            }
        }
    } else if (j0 == 0 && j1 == S) {
        store_contig<R, S>(qout + s0, st.q);
        store_contig<R, S>(pout + s0, st.p);
        if constexpr (KAHAN) {
            store_contig<C, S>(cqout + s0, st.cq);
            store_contig<C, S>(cpout + s0, st.cp);
        }
    } else {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (j >= j0 && j < j1) {
                const int64_t g = s0 + j;
                qout[g] = st.q[j];
                pout[g] = st.p[j];
                if constexpr (KAHAN) {
                    cqout[g] = st.cq[j];
                    cpout[g] = st.cp[j];
                }
            }
        }
    }
}

// Device-coherent stores of one array of a wavefront's kept sites through a
// staging area in LDS of 64*S values. Lane l holds S consecutive values, so
// unstaged, store m of the wavefront writes 16 bytes at every 16*S-th byte:
// half of each 32-byte sector, and each store counts as a whole sector in
// memory (those stores moved twice their bytes). Staged, lane l first puts
// its values in its own S slots; then store m of lane l moves piece 64*m + l
// (16 bytes), so one store instruction covers 1 KB of consecutive addresses.
// `keep(pos)` says which cluster-local positions are written; a piece whose
// values are all kept goes as one 16-byte store, a piece cut by the end of
// the kept positions (the end of a chain that is not a multiple of 4 sites)
// value by value. `out_e0` is the array at the cluster origin and `bytes`
// the window the buffer resource spans (a store beyond it is dropped). Only
// this wavefront's lanes touch `stage`, so wavefront-scope ordering suffices
// between its write and reads.
template <class R, int S, class Keep>
__device__ __forceinline__ void store_staged(R *stage, const R (&v)[S], R *out_e0, int bytes,
                                             int lane, int wlo, Keep keep) {
    constexpr int P = 16 / static_cast<int>(sizeof(R));  // values per 16-byte piece
    static_assert(S % P == 0, "whole 16-byte pieces per lane");
    using U4 = __attribute__((ext_vector_type(4))) unsigned;
    struct Piece {
        R x[P];
    };
#pragma unroll
    for (int m = 0; m < S / P; ++m) {
        Piece pc;
#pragma unroll
        for (int t = 0; t < P; ++t) pc.x[t] = v[P * m + t];
        *reinterpret_cast<U4 *>(stage + lane * S + P * m) = __builtin_bit_cast(U4, pc);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const __amdgpu_buffer_rsrc_t r = window_rsrc(out_e0, bytes);
#pragma unroll
    for (int m = 0; m < S / P; ++m) {
        const int c = 64 * m + lane;   // piece of this wavefront
        const int loc = wlo + P * c;   // cluster-local position of its first value
        const U4 x = *reinterpret_cast<const U4 *>(stage + P * c);
        bool all = true, any = false;
#pragma unroll
        for (int t = 0; t < P; ++t) {
            const bool k = keep(loc + t);
            all = all && k;
            any = any || k;
        }
        if (all) {
            __builtin_amdgcn_raw_buffer_store_b128(x, r, loc * static_cast<int>(sizeof(R)), 0,
                                                   kDeviceCoherent);
        } else if (any) {
            const Piece pc = __builtin_bit_cast(Piece, x);
#pragma unroll
            for (int t = 0; t < P; ++t)
                if (keep(loc + t)) store_coherent(out_e0 + loc + t, pc.x[t]);
        }
    }
    // the next array reuses the staging area
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One cluster pass: the cluster holds sites [e0, e0 + 64*S*W) of the
// unwrapped ring (wrapped mod n on load), advances them `ksteps` steps and
// stores the sites at cluster-local positions [halo, halo + keep). The wrong
// values that enter at the cluster edges move 2*range sites per step: dq/dt =
// p is local, so a coordinate error reaches the force of the next site only
// every second stage. The caller guarantees halo >= 2*range*ksteps and
// halo + keep <= 64*S*W, so the stored sites are exact. All wavefronts of
// the cluster must call this together.
template <int M, class R, bool KAHAN, int S, int W, int WPB, bool COH = false, class C = float>
__device__ __forceinline__ void run_cluster(const StateRef &in, const StateRef &out, int64_t n,
                                            int64_t e0, int64_t halo, int64_t keep, int ksteps,
                                            double dt, SlotsOf<M, R, W, WPB> *slots, int lane,
                                            int wib, int wic, int prio_total = 0,
                                            R *stage = nullptr) {
    constexpr int E = 64 * S * W;
    const int lo = (wic * 64 + lane) * S;
    const int64_t s0 = e0 + lo;
    LaneState<R, KAHAN, S, C> st;
    load_lane<R, KAHAN, S, COH, C>(st, in, n, s0, e0 >= 0 && e0 + E <= n);
    const StepConsts<R, KAHAN> c(dt);
    R Q[S], X[S], s[S], a[S];  // stage argument and the values site_update carries
    if constexpr (W == 1) {
        // one-wavefront clusters (short chains, the whole launch resident at
        // once): issue priority by progress when prio_total > 0
        steps_by_progress(0, ksteps, prio_total, [&] {
            any_lane_stage<M, S, 1, W, WPB>(Q, X, st.q, st.p, s, a, c, slots, lane, wib, wic, 0);
            any_lane_stage<M, S, 2, W, WPB>(Q, X, st.q, st.p, s, a, c, slots, lane, wib, wic, 1);
            any_lane_stage<M, S, 3, W, WPB>(Q, X, st.q, st.p, s, a, c, slots, lane, wib, wic, 0);
            any_lane_stage<M, S, 4, W, WPB>(Q, X, st.q, st.p, s, a, c, slots, lane, wib, wic, 1);
            if constexpr (KAHAN)
                final_update_kahan<S>(st.q, st.p, st.cq, st.cp, s, a, c);
            else
                final_update<S>(st.q, st.p, s, a, c);
        });
    } else {
        for (int k = 0; k < ksteps; ++k) {
            any_lane_stage<M, S, 1, W, WPB>(Q, X, st.q, st.p, s, a, c, slots, lane, wib, wic, 0);
            any_lane_stage<M, S, 2, W, WPB>(Q, X, st.q, st.p, s, a, c, slots, lane, wib, wic, 1);
            any_lane_stage<M, S, 3, W, WPB>(Q, X, st.q, st.p, s, a, c, slots, lane, wib, wic, 0);
            any_lane_stage<M, S, 4, W, WPB>(Q, X, st.q, st.p, s, a, c, slots, lane, wib, wic, 1);
            if constexpr (KAHAN)
                final_update_kahan<S>(st.q, st.p, st.cq, st.cp, s, a, c);
            else
                final_update<S>(st.q, st.p, s, a, c);
        }
    }
    // The store's per-lane offsets are formed again from the lane id after
    // the step loop. The empty asm hides that the id is the one used for the
    // load, so the compiler cannot keep 64-bit offsets and addresses from
    // before the loop live through it (in the batch kernel they held ten
    // registers and pushed it past 128).
    int lane_s = lane;
    asm volatile("" : "+v"(lane_s));
    if constexpr (COH && (!KAHAN || std::is_same<C, R>::value) && (S * sizeof(R)) % 16 == 0) {
        if (stage) {
            // kept sites never wrap, and the chain ends at n: the kept range
            // in cluster-local positions, and each array at the cluster origin
            const int kl = static_cast<int>(halo);
            const int kh = static_cast<int>(halo + keep < n - e0 ? halo + keep : n - e0);
            const int wlo = wic * 64 * S;
            constexpr int bytes = E * static_cast<int>(sizeof(R));
            auto kept = [kl, kh](int pos) { return pos >= kl && pos < kh; };
            store_staged<R, S>(stage, st.q, static_cast<R *>(out.q) + e0, bytes, lane_s, wlo, kept);
            store_staged<R, S>(stage, st.p, static_cast<R *>(out.p) + e0, bytes, lane_s, wlo, kept);
            if constexpr (KAHAN) {
                store_staged<R, S>(stage, st.cq, static_cast<R *>(out.cq) + e0, bytes, lane_s, wlo,
                                   kept);
                store_staged<R, S>(stage, st.cp, static_cast<R *>(out.cp) + e0, bytes, lane_s, wlo,
                                   kept);
            }
            return;
        }
    }
    const int lo_s = (wic * 64 + lane_s) * S;
    store_lane<R, KAHAN, S, COH, C>(st, out, n, e0 + lo_s, lo_s, halo, halo + keep, E);
}

// Whole-ring resident run by a block of T threads: thread t owns sites
// t + T*j (j < SPT, n <= T*SPT). The stage argument of every site is
// published in LDS (`lds` holds 2*n values, two buffers used in turn, one
// barrier per stage); the state and the values carried between stages stay
// in registers.
// `out` may equal `in`: every load happens before the first store.
template <int M, class R, bool KAHAN, int T, int SPT>
__device__ __forceinline__ void run_resident(const StateRef &in, const StateRef &out, int n,
                                             int64_t nsteps, double dt, R *lds) {
    R *buf0 = lds;
    R *buf1 = lds + n;
    const int t = threadIdx.x;
    const R *qin = static_cast<const R *>(in.q);
    const R *pin = static_cast<const R *>(in.p);
    R q[SPT], p[SPT], Q[SPT], X[SPT], s[SPT], a[SPT];  // Q: own stage argument
    float cq[KAHAN ? SPT : 1], cp[KAHAN ? SPT : 1];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int i = t + T * j;
        if (i < n) {
            q[j] = qin[i];
            p[j] = pin[i];
            if constexpr (KAHAN) {
                cq[j] = static_cast<const float *>(in.cq)[i];
                cp[j] = static_cast<const float *>(in.cp)[i];
            }
            buf0[i] = q[j];
            Q[j] = q[j];
        }
    }
    __syncthreads();

    const StepConsts<R, KAHAN> c(dt);
    for (int64_t st = 0; st < nsteps; ++st) {
        // stage s reads its argument from `cur` and publishes the next one
        // (after stage 4: the new coordinates) in `nxt`
#pragma unroll
        for (int stage = 1; stage <= 4; ++stage) {
            const R *cur = (stage & 1) ? buf0 : buf1;
            R *nxt = (stage & 1) ? buf1 : buf0;
#pragma unroll
            for (int j = 0; j < SPT; ++j) {
                const int i = t + T * j;
                if (i < n) {
                    const int im = (i == 0) ? n - 1 : i - 1;
                    const int ip = (i == n - 1) ? 0 : i + 1;
                    const R Qm = cur[im], Qj = Q[j], Qp = cur[ip];
                    R Qn = Qj;
                    if (stage == 1) {
                        stage_one<M, 1, R>(Qm, Qj, Qp, q[j], p[j], X[j], s[j], a[j], Qn, c);
                    } else if (stage == 2) {
                        stage_one<M, 2, R>(Qm, Qj, Qp, q[j], p[j], X[j], s[j], a[j], Qn, c);
                    } else if (stage == 3) {
                        stage_one<M, 3, R>(Qm, Qj, Qp, q[j], p[j], X[j], s[j], a[j], Qn, c);
                    } else {
                        stage_one<M, 4, R>(Qm, Qj, Qp, q[j], p[j], X[j], s[j], a[j], Qn, c);
                        site_final<R, KAHAN, float>(q[j], p[j], cq[KAHAN ? j : 0],
                                                    cp[KAHAN ? j : 0], s[j], a[j], c);
                        Qn = q[j];
                    }
                    nxt[i] = Qn;
                    Q[j] = Qn;
                }
            }
            __syncthreads();
        }
    }

    R *qout = static_cast<R *>(out.q);
    R *pout = static_cast<R *>(out.p);
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int i = t + T * j;
        if (i < n) {
            qout[i] = q[j];
            pout[i] = p[j];
            if constexpr (KAHAN) {
                static_cast<float *>(out.cq)[i] = cq[j];
                static_cast<float *>(out.cp)[i] = cp[j];
            }
        }
    }
}

// Workgroups of `Kernel` (blocks of `threads`) the current device holds at
// once; 0 if the query fails. Cached per device.
template <auto Kernel>
int resident_blocks(int threads) {
    static std::atomic<int> cached[64];  // handles on different threads may ask at once
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int v = cached[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, Kernel, threads, 0) != hipSuccess)
            return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        v = per_cu * cus;
        cached[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

}  // namespace chainrk4
