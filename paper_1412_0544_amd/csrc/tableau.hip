// tableau.hip -- the fused cluster pass for any explicit Runge-Kutta method
// given by its Butcher tableau (Sec. 2.2 Eq. 3-5 with general coefficients;
// Sec. 2 notes the cluster technique carries over to every explicit scheme).
//
// The cluster, the loads, the stores and the lane exchange are those of the
// classical-RK4 kernel; only the stage arithmetic differs. Every stage keeps
// its slope k_j = (P_j, F(Q_j)) in registers, so the stage argument
//   (Q_j, P_j) = (q, p) + dt * sum_{m<j} a[j][m] k_m
// and the final combination (q, p) + dt * sum_m b[m] k_m can use any
// coefficients. The tableau arrives as a kernel argument; SMAX (4 or 8) bounds
// the stage count at compile time so the slopes stay in registers.
#include "cluster.hpp"

namespace chainrk4 {
namespace {

// Forces F_j at the stage argument Q of this lane's S sites; the neighbour
// coordinates cross lanes and wavefronts as in lane_stage / lane_stage_nnn,
// with the same operations, so edge bond terms are bitwise those of the
// neighbour.
template <int M, int S, int W, int WPB, class R>
__device__ __forceinline__ void lane_force(const R (&Q)[S], R (&F)[S], SlotsOf<M, R, WPB> *slots,
                                           int lane, int wib, int wic, int parity) {
    using Ops = ModelOps<M, R>;
    if constexpr (coupling_range<M>() == 1) {
        const R first = Q[0], last = Q[S - 1];
        R right = from_right(first);
        if constexpr (W > 1) {
            if (lane == 0) slots->first[parity][wib] = first;
            if (lane == 63) slots->last[parity][wib] = last;
            __syncthreads();
            if (lane == 63 && wic + 1 < W) right = slots->first[parity][wib + 1];
        }
        const R brS = Ops::bond(right - last);
        R bl = from_left(brS);
        if constexpr (W > 1) {
            if (lane == 0 && wic > 0) bl = Ops::bond(first - slots->last[parity][wib - 1]);
        }
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const R br = (j + 1 < S) ? Ops::bond(Q[j + 1] - Q[j]) : brS;
            F[j] = site_force<M, R>(bl, br, Q[j]);
            bl = br;
        }
    } else {
        const R f0 = Q[0], f1 = Q[1], l1 = Q[S - 2], l0 = Q[S - 1];
        R r0 = from_right(f0), r1 = from_right(f1);
        if constexpr (W > 1) {
            if (lane == 0) {
                slots->first[parity][0][wib] = f0;
                slots->first[parity][1][wib] = f1;
            }
            if (lane == 63) {
                slots->last[parity][0][wib] = l0;
                slots->last[parity][1][wib] = l1;
            }
            __syncthreads();
            if (lane == 63 && wic + 1 < W) {
                r0 = slots->first[parity][0][wib + 1];
                r1 = slots->first[parity][1][wib + 1];
            }
        }
        const R b1rS = Ops::bond(r0 - l0), b2rS2 = Ops::bond(r0 - l1), b2rS1 = Ops::bond(r1 - l0);
        R b1l = from_left(b1rS), b2lo = from_left(b2rS2), b2hi = from_left(b2rS1);
        if constexpr (W > 1) {
            if (lane == 0 && wic > 0) {
                const R L0 = slots->last[parity][0][wib - 1];
                const R L1 = slots->last[parity][1][wib - 1];
                b1l = Ops::bond(f0 - L0);
                b2lo = Ops::bond(f0 - L1);
                b2hi = Ops::bond(f1 - L0);
            }
        }
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const R b1r = (j + 1 < S) ? Ops::bond(Q[j + 1] - Q[j]) : b1rS;
            const R b2r = (j + 2 < S) ? Ops::bond(Q[j + 2] - Q[j]) : ((j + 2 == S) ? b2rS2 : b2rS1);
            F[j] = site_force2<M, R>(b1l, b1r, b2lo, b2r, Q[j]);
            b1l = b1r;
            b2lo = b2hi;
            b2hi = b2r;
        }
    }
}

constexpr int tab_block_threads(int W) { return W == 1 ? kFusedThreads : 64 * W; }

template <int M, class R, bool KAHAN, int S, int W, int SMAX>
__global__ __launch_bounds__(tab_block_threads(W)) void tableau_kernel(FusedPass a, TabArgs t) {
    constexpr int WPB = tab_block_threads(W) / 64;
    constexpr int CPB = WPB / W;
    constexpr int E = 64 * S * W;
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int wic = wib % W;
    const int64_t cluster = static_cast<int64_t>(blockIdx.x) * CPB + wib / W;
    __shared__ SlotsOf<M, R, WPB> slots;
    if (cluster >= a.waves) return;  // W = 1 only (a W > 1 grid has no extra blocks)
    const int64_t e0 = cluster * a.tile - a.halo;
    const int lo = (wic * 64 + lane) * S;
    const int64_t s0 = e0 + lo;
    LaneState<R, KAHAN, S> st;
    load_lane<R, KAHAN, S>(st, a.in, a.n, s0, e0 >= 0 && e0 + E <= a.n);
    const R dt = static_cast<R>(a.dt);
    const R dtlo = static_cast<R>(a.dt - static_cast<double>(dt));  // dt - R(dt)
    const int s = t.stages;
    // kq[m] holds P_m (the q part of k_m) for m >= 1; the q part of k_0 is p
    R kq[SMAX][S], kp[SMAX][S], Q[S], fq[S], fp[S];
    int parity = 0;
    for (int k = 0; k < a.ksteps; ++k) {
#pragma unroll
        for (int j = 0; j < SMAX; ++j) {
            if (j >= s) break;  // uniform: the stage count is a kernel argument
            if (j == 0) {
                lane_force<M, S, W, WPB>(st.q, kp[0], &slots, lane, wib, wic, parity);
            } else {
#pragma unroll
                for (int i = 0; i < S; ++i) {
                    R sq = static_cast<R>(0), sp = static_cast<R>(0);
#pragma unroll
                    for (int m = 0; m < j; ++m) {
                        const R c = static_cast<R>(t.a[j][m]);
                        sq = fma_r(c, m == 0 ? st.p[i] : kq[m][i], sq);
                        sp = fma_r(c, kp[m][i], sp);
                    }
                    Q[i] = fma_r(dt, sq, st.q[i]);
                    kq[j][i] = fma_r(dt, sp, st.p[i]);
                }
                lane_force<M, S, W, WPB>(Q, kp[j], &slots, lane, wib, wic, parity);
            }
            parity ^= 1;
            // the final combination, accumulated stage by stage in stage order
            const R bj = static_cast<R>(t.b[j]);
#pragma unroll
            for (int i = 0; i < S; ++i) {
                const R kqj = j == 0 ? st.p[i] : kq[j][i];
                fq[i] = j == 0 ? bj * kqj : fma_r(bj, kqj, fq[i]);
                fp[i] = j == 0 ? bj * kp[0][i] : fma_r(bj, kp[j][i], fp[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if constexpr (KAHAN) {
                kahan_step(st.q[i], st.cq[i], fq[i], dt, dtlo);
                kahan_step(st.p[i], st.cp[i], fp[i], dt, dtlo);
            } else {
                st.q[i] = fma_r(dt, fq[i], st.q[i]);
                st.p[i] = fma_r(dt, fp[i], st.p[i]);
            }
        }
    }
    store_lane<R, KAHAN, S>(st, a.out, a.n, s0, lo, a.halo, a.halo + a.tile);
}

template <int M, class R, bool KAHAN, int S, int W, int SMAX>
hipError_t tab_launch_one(const FusedPass &a, const TabArgs &t, hipStream_t st) {
    constexpr int T = tab_block_threads(W);
    constexpr int cpb = T / 64 / W;
    const int64_t blocks64 = (a.waves + cpb - 1) / cpb;
    if (blocks64 <= 0 || blocks64 > 0x7fffffff) return hipErrorInvalidValue;
    tableau_kernel<M, R, KAHAN, S, W, SMAX><<<dim3(static_cast<unsigned>(blocks64)), dim3(T), 0, st>>>(a, t);
    return hipGetLastError();
}

template <int M, class R, bool KAHAN>
hipError_t tab_dispatch(int s, int w, const FusedPass &a, const TabArgs &t, hipStream_t st) {
    if (t.stages <= 4) {
        if (s == 4) return w == 1 ? tab_launch_one<M, R, KAHAN, 4, 1, 4>(a, t, st)
                          : w == 4 ? tab_launch_one<M, R, KAHAN, 4, 4, 4>(a, t, st)
                                   : hipErrorInvalidValue;
        if (s == 8) return w == 1 ? tab_launch_one<M, R, KAHAN, 8, 1, 4>(a, t, st)
                          : w == 4 ? tab_launch_one<M, R, KAHAN, 8, 4, 4>(a, t, st)
                                   : hipErrorInvalidValue;
        return hipErrorInvalidValue;
    }
    if (t.stages <= kMaxStages && s == 4)
        return w == 1 ? tab_launch_one<M, R, KAHAN, 4, 1, kMaxStages>(a, t, st)
             : w == 4 ? tab_launch_one<M, R, KAHAN, 4, 4, kMaxStages>(a, t, st)
                      : hipErrorInvalidValue;
    return hipErrorInvalidValue;
}

template <int M>
hipError_t tab_dispatch_prec(int prec, int s, int w, const FusedPass &a, const TabArgs &t,
                             hipStream_t st) {
    return prec == 0 ? tab_dispatch<M, double, false>(s, w, a, t, st)
                     : tab_dispatch<M, float, true>(s, w, a, t, st);
}

constexpr int kNaiveTabThreads = 256;

// Stage j of the per-stage implementation at site i: the slope k_j at the
// stage argument (Qj from `arg`, with its neighbours; Pj), then the next stage
// argument, or the final combination in place. Same per-site operation order
// as tableau_kernel, so both give identical bits.
template <int M, class R, bool KAHAN>
__global__ __launch_bounds__(kNaiveTabThreads) void naive_tab_stage(StateRef y, NaiveTabBufs b,
                                                                    const R *argq, const R *argp,
                                                                    R *nextq, R *nextp, int j,
                                                                    int64_t n, double dt_,
                                                                    TabArgs t) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kNaiveTabThreads + threadIdx.x;
    if (i >= n) return;
    using Ops = ModelOps<M, R>;
    const R dt = static_cast<R>(dt_);
    const R dtlo = static_cast<R>(dt_ - static_cast<double>(dt));  // dt - R(dt)
    R *yq = static_cast<R *>(y.q);
    R *yp = static_cast<R *>(y.p);
    const R Qj = argq[i];
    const R Pj = argp[i];
    R F;
    if constexpr (coupling_range<M>() == 2) {
        F = site_force2<M, R>(Ops::bond(Qj - argq[wrap_index(i - 1, n)]),
                              Ops::bond(argq[wrap_index(i + 1, n)] - Qj),
                              Ops::bond(Qj - argq[wrap_index(i - 2, n)]),
                              Ops::bond(argq[wrap_index(i + 2, n)] - Qj), Qj);
    } else {
        F = site_force<M, R>(Ops::bond(Qj - argq[wrap_index(i - 1, n)]),
                             Ops::bond(argq[wrap_index(i + 1, n)] - Qj), Qj);
    }
    const R qi = yq[i], pi = yp[i];
    // slope m at this site: (P_m, F_m); stage j's comes from registers
    auto kqm = [&](int m) -> R {
        return m == j ? Pj : (m == 0 ? pi : static_cast<const R *>(b.kq[m])[i]);
    };
    auto kpm = [&](int m) -> R { return m == j ? F : static_cast<const R *>(b.kp[m])[i]; };
    if (j + 1 < t.stages) {
        if (j > 0) static_cast<R *>(b.kq[j])[i] = Pj;
        static_cast<R *>(b.kp[j])[i] = F;
        R sq = static_cast<R>(0), sp = static_cast<R>(0);
        for (int m = 0; m <= j; ++m) {
            const R c = static_cast<R>(t.a[j + 1][m]);
            sq = fma_r(c, kqm(m), sq);
            sp = fma_r(c, kpm(m), sp);
        }
        nextq[i] = fma_r(dt, sq, qi);
        nextp[i] = fma_r(dt, sp, pi);
    } else {
        R fq = static_cast<R>(t.b[0]) * kqm(0);
        R fp = static_cast<R>(t.b[0]) * kpm(0);
        for (int m = 1; m < t.stages; ++m) {
            const R c = static_cast<R>(t.b[m]);
            fq = fma_r(c, kqm(m), fq);
            fp = fma_r(c, kpm(m), fp);
        }
        if constexpr (KAHAN) {
            R q1 = qi, p1 = pi;
            float *ycq = static_cast<float *>(y.cq), *ycp = static_cast<float *>(y.cp);
            float cq = ycq[i], cp = ycp[i];
            kahan_step(q1, cq, fq, dt, dtlo);
            kahan_step(p1, cp, fp, dt, dtlo);
            yq[i] = q1;
            yp[i] = p1;
            ycq[i] = cq;
            ycp[i] = cp;
        } else {
            yq[i] = fma_r(dt, fq, qi);
            yp[i] = fma_r(dt, fp, pi);
        }
    }
}

template <int M, class R, bool KAHAN>
hipError_t naive_tab_dispatch(StateRef y, const NaiveTabBufs &b, int64_t n, double dt,
                              const TabArgs &t, hipStream_t st) {
    const int64_t blocks = (n + kNaiveTabThreads - 1) / kNaiveTabThreads;
    if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(blocks)), block(kNaiveTabThreads);
    const R *aq = static_cast<const R *>(y.q), *ap = static_cast<const R *>(y.p);
    if (t.stages == 1) {
        // the only stage would read neighbours of q while writing q: read a copy
        hipError_t e = hipMemcpyAsync(b.qa, y.q, n * sizeof(R), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
        aq = static_cast<const R *>(b.qa);
    }
    for (int j = 0; j < t.stages; ++j) {
        R *nq = static_cast<R *>(j % 2 == 0 ? b.qa : b.qb);
        R *np = static_cast<R *>(j % 2 == 0 ? b.pa : b.pb);
        if (t.stages == 1) nq = np = nullptr;
        naive_tab_stage<M, R, KAHAN><<<grid, block, 0, st>>>(y, b, aq, ap, nq, np, j, n, dt, t);
        aq = nq;
        ap = np;
    }
    return hipGetLastError();
}

template <int M>
hipError_t naive_tab_prec(int prec, StateRef y, const NaiveTabBufs &b, int64_t n, double dt,
                          const TabArgs &t, hipStream_t st) {
    return prec == 0 ? naive_tab_dispatch<M, double, false>(y, b, n, dt, t, st)
                     : naive_tab_dispatch<M, float, true>(y, b, n, dt, t, st);
}

}  // namespace

hipError_t launch_naive_tableau_step(int model, int prec, StateRef y, const NaiveTabBufs &b,
                                     int64_t n, double dt, const TabArgs &t, hipStream_t st) {
    if (t.stages < 1 || t.stages > kMaxStages) return hipErrorInvalidValue;
    switch (model) {
    case kQuartic: return naive_tab_prec<kQuartic>(prec, y, b, n, dt, t, st);
    case kHarmonic: return naive_tab_prec<kHarmonic>(prec, y, b, n, dt, t, st);
    case kQuarticNNN: return naive_tab_prec<kQuarticNNN>(prec, y, b, n, dt, t, st);
    case kHarmonicNNN: return naive_tab_prec<kHarmonicNNN>(prec, y, b, n, dt, t, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tableau(int model, int prec, int s, int w, const FusedPass &a, const TabArgs &t,
                          hipStream_t st) {
    if (t.stages < 1 || t.stages > kMaxStages) return hipErrorInvalidValue;
    switch (model) {
    case kQuartic: return tab_dispatch_prec<kQuartic>(prec, s, w, a, t, st);
    case kHarmonic: return tab_dispatch_prec<kHarmonic>(prec, s, w, a, t, st);
    case kQuarticNNN: return tab_dispatch_prec<kQuarticNNN>(prec, s, w, a, t, st);
    case kHarmonicNNN: return tab_dispatch_prec<kHarmonicNNN>(prec, s, w, a, t, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace chainrk4
