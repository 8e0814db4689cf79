// tableau.hip -- the fused cluster pass for any explicit Runge-Kutta method
// given by its Butcher tableau (Sec. 2.2 Eq. 3-5 with general coefficients;
// Sec. 2 notes the cluster technique carries over to every explicit scheme).
//
// The cluster, the loads, the stores and the lane exchange are those of the
// classical-RK4 kernel; only the stage arithmetic differs. For dq/dt = p,
// dp/dt = F(q) the q slopes are the p stage values P_m = p + h sum_l a_ml F_l,
// so (exact algebra on Eq. 3-5 with general coefficients)
//   Q_j = q + h c_j p + h^2 sum_l (A^2)_jl F_l,        c_j = sum_m a_jm,
//   q'  = q + h (sum_m b_m) p + h^2 sum_l (b^T A)_l F_l,
//   p'  = p + h sum_m b_m F_m,
// and only the forces F_l of the stages are kept (in registers). (A^2)_jl is
// zero for l >= j - 1 and (b^T A)_l for the last stage, so those terms are not
// formed. The host derives the coefficients, scaled by the step, in FP64 (TabArgs);
// SMAX (4, 6 or 8) bounds the stage count at compile time.
#include "cluster.hpp"

namespace chainrk4 {
namespace {

// Forces F_j at the stage argument Q of this lane's S sites; the bond terms
// that join two lanes come from the same exchange as in the RK4 cluster pass
// (edge_bonds / edge_bonds2), so they are bitwise those of the neighbour.
template <int M, int S, int W, int WPB, class R>
__device__ __forceinline__ void lane_force(const R (&Q)[S], R (&F)[S],
                                           SlotsOf<M, R, W, WPB> *slots, int lane, int wib,
                                           int wic, int parity) {
    using Ops = ModelOps<M, R>;
    if constexpr (coupling_range<M>() == 1) {
        R bl, brS;
        edge_bonds<M, W, WPB>(Q[0], Q[S - 1], slots, lane, wib, wic, parity, bl, brS);
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const R br = (j + 1 < S) ? Ops::bond(Q[j + 1] - Q[j]) : brS;
            F[j] = site_force<M, R>(bl, br, Q[j]);
            bl = br;
        }
    } else {
        R b1l, b2lo, b2hi, b1rS, b2rS2, b2rS1;
        edge_bonds2<M, W, WPB>(Q[0], Q[1], Q[S - 1], Q[S - 2], slots, lane, wib, wic, parity, b1l,
                               b2lo, b2hi, b1rS, b2rS2, b2rS1);
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

// A coefficient as two parts in the working precision: hi = R(x), lo = R(x - hi).
// For FP64 the second part is not used.
template <class R>
struct Coef {
    R hi, lo;
    __device__ __forceinline__ explicit Coef(double x)
        : hi(static_cast<R>(x)), lo(static_cast<R>(x - static_cast<double>(static_cast<R>(x)))) {}
};

// acc += x * F. FP64 rounds once; the compensated FP32 form takes x in two
// parts, since a coefficient rounded once to FP32 would scale the same term
// of every step alike (an error the carry of the update cannot undo). The
// product (hi + lo) F is rounded once before it meets the sum: acc + lo F
// would round back to acc, losing the small part in every step.
template <class R, bool KAHAN>
__device__ __forceinline__ R coef_fma(const Coef<R> &x, R F, R acc, bool first) {
    if constexpr (KAHAN) {
        const R t = fma_r(x.hi, F, x.lo * F);
        return first ? t : acc + t;
    } else {
        return first ? x.hi * F : fma_r(x.hi, F, acc);
    }
}

// The stage argument Q_j = q + hc_j p + sum_l g_jl F_l at one site, the sum
// taken in stage order. FP64 accumulates into q. The compensated FP32 form
// takes hc_j in two parts and forms the increment apart, adding it to q last:
// a factor rounded once to FP32 would offset every stage argument alike (an
// energy term of the same sign in every step), and its small part added to q
// directly would round away.
template <class R, bool KAHAN>
__device__ __forceinline__ R stage_start(const Coef<R> &hc, R q, R p) {
    if constexpr (KAHAN)
        return fma_r(hc.hi, p, hc.lo * p);
    else
        return fma_r(hc.hi, p, q);
}
template <class R, bool KAHAN>
__device__ __forceinline__ R stage_end(R x, R q) {
    if constexpr (KAHAN)
        return q + x;
    else
        return x;
}

template <int M, class R, bool KAHAN, int S, int W, int SMAX>
__global__ __launch_bounds__(tab_block_threads(W)) void tableau_kernel(FusedPass a, TabArgs t) {
    constexpr int WPB = tab_block_threads(W) / 64;
    constexpr int CPB = WPB / W;
    constexpr int E = 64 * S * W;
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int wic = wib % W;
    const int64_t cluster = static_cast<int64_t>(blockIdx.x) * CPB + wib / W;
    __shared__ SlotsOf<M, R, W, WPB> slots;
    if (cluster >= a.waves) return;  // W = 1 only (a W > 1 grid has no extra blocks)
    const int64_t e0 = cluster * a.tile - a.halo;
    const int lo = (wic * 64 + lane) * S;
    const int64_t s0 = e0 + lo;
    LaneState<R, KAHAN, S> st;
    load_lane<R, KAHAN, S>(st, a.in, a.n, s0, e0 >= 0 && e0 + E <= a.n);
    const int s = t.stages;
    R F[SMAX][S], Q[S], fq[S], fp[S];
    int parity = 0;
    for (int k = 0; k < a.ksteps; ++k) {
#pragma unroll
        for (int j = 0; j < SMAX; ++j) {
            if (j >= s) break;  // uniform: the stage count is a kernel argument
            if (j == 0) {
                lane_force<M, S, W, WPB>(st.q, F[0], &slots, lane, wib, wic, parity);
            } else {
                const Coef<R> hc(t.hc[j]);
#pragma unroll
                for (int i = 0; i < S; ++i) {
                    R x = stage_start<R, KAHAN>(hc, st.q[i], st.p[i]);
#pragma unroll
                    for (int l = 0; l + 1 < j; ++l) x = fma_r(static_cast<R>(t.g[j][l]), F[l][i], x);
                    Q[i] = stage_end<R, KAHAN>(x, st.q[i]);
                }
                lane_force<M, S, W, WPB>(Q, F[j], &slots, lane, wib, wic, parity);
            }
            parity ^= 1;
            // the final combination, accumulated stage by stage in stage order
            // (w of the last stage is zero, which adds nothing: no branch)
            const Coef<R> hb(t.hb[j]), w(t.w[j]);
#pragma unroll
            for (int i = 0; i < S; ++i) {
                fp[i] = coef_fma<R, KAHAN>(hb, F[j][i], fp[i], j == 0);
                fq[i] = coef_fma<R, KAHAN>(w, F[j][i], fq[i], j == 0);
            }
        }
        const Coef<R> hsb(t.hsb);
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if constexpr (KAHAN) {
                kahan_finish(st.q[i], st.cq[i],
                             fma_r(hsb.hi, st.p[i], fma_r(hsb.lo, st.p[i], fq[i] - st.cq[i])));
                kahan_finish(st.p[i], st.cp[i], fp[i] - st.cp[i]);
            } else {
                st.q[i] = fma_r(hsb.hi, st.p[i], st.q[i]) + fq[i];
                st.p[i] = st.p[i] + fp[i];
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
    // 5 or 6 stages (Dormand-Prince 5 without its last, first-same-as-last
    // stage): registers for 6 forces instead of 8, one more wavefront per SIMD
    if (t.stages <= 6 && s == 4)
        return w == 1 ? tab_launch_one<M, R, KAHAN, 4, 1, 6>(a, t, st)
             : w == 4 ? tab_launch_one<M, R, KAHAN, 4, 4, 6>(a, t, st)
                      : hipErrorInvalidValue;
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

// Stage j of the per-stage implementation at site i: the force F_j at the
// stage argument (from `arg`, with its neighbours), kept in memory for the
// later stages, then the next stage argument, or the final combination in
// place. Same per-site operation order as tableau_kernel, so both give
// identical bits.
template <int M, class R, bool KAHAN>
__global__ __launch_bounds__(kNaiveTabThreads) void naive_tab_stage(StateRef y, NaiveTabBufs b,
                                                                    const R *arg, R *next, int j,
                                                                    int64_t n, TabArgs t) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kNaiveTabThreads + threadIdx.x;
    if (i >= n) return;
    using Ops = ModelOps<M, R>;
    R *yq = static_cast<R *>(y.q);
    R *yp = static_cast<R *>(y.p);
    const R Qj = arg[i];
    R Fj;
    if constexpr (coupling_range<M>() == 2) {
        Fj = site_force2<M, R>(Ops::bond(Qj - arg[wrap_index(i - 1, n)]),
                               Ops::bond(arg[wrap_index(i + 1, n)] - Qj),
                               Ops::bond(Qj - arg[wrap_index(i - 2, n)]),
                               Ops::bond(arg[wrap_index(i + 2, n)] - Qj), Qj);
    } else {
        Fj = site_force<M, R>(Ops::bond(Qj - arg[wrap_index(i - 1, n)]),
                              Ops::bond(arg[wrap_index(i + 1, n)] - Qj), Qj);
    }
    const R qi = yq[i], pi = yp[i];
    // force of stage m at this site; stage j's comes from registers
    auto Fm = [&](int m) -> R { return m == j ? Fj : static_cast<const R *>(b.kp[m])[i]; };
    const int s = t.stages;
    if (j + 1 < s) {
        static_cast<R *>(b.kp[j])[i] = Fj;
        R x = stage_start<R, KAHAN>(Coef<R>(t.hc[j + 1]), qi, pi);
        for (int l = 0; l < j; ++l) x = fma_r(static_cast<R>(t.g[j + 1][l]), Fm(l), x);
        next[i] = stage_end<R, KAHAN>(x, qi);
    } else {
        R fq = static_cast<R>(0), fp = static_cast<R>(0);
        for (int m = 0; m < s; ++m) {
            const Coef<R> hb(t.hb[m]), w(t.w[m]);
            const R f = Fm(m);
            fp = coef_fma<R, KAHAN>(hb, f, fp, m == 0);
            fq = coef_fma<R, KAHAN>(w, f, fq, m == 0);
        }
        const Coef<R> hsb(t.hsb);
        if constexpr (KAHAN) {
            R q1 = qi, p1 = pi;
            float *ycq = static_cast<float *>(y.cq), *ycp = static_cast<float *>(y.cp);
            float cq = ycq[i], cp = ycp[i];
            kahan_finish(q1, cq, fma_r(hsb.hi, pi, fma_r(hsb.lo, pi, fq - cq)));
            kahan_finish(p1, cp, fp - cp);
            yq[i] = q1;
            yp[i] = p1;
            ycq[i] = cq;
            ycp[i] = cp;
        } else {
            yq[i] = fma_r(hsb.hi, pi, qi) + fq;
            yp[i] = pi + fp;
        }
    }
}

template <int M, class R, bool KAHAN>
hipError_t naive_tab_dispatch(StateRef y, const NaiveTabBufs &b, int64_t n,
                              double /* dt: already in the coefficients of t */,
                              const TabArgs &t, hipStream_t st) {
    const int64_t blocks = (n + kNaiveTabThreads - 1) / kNaiveTabThreads;
    if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(blocks)), block(kNaiveTabThreads);
    const R *arg = static_cast<const R *>(y.q);
    if (t.stages == 1) {
        // the only stage would read neighbours of q while writing q: read a copy
        hipError_t e = hipMemcpyAsync(b.qa, y.q, n * sizeof(R), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
        arg = static_cast<const R *>(b.qa);
    }
    for (int j = 0; j < t.stages; ++j) {
        R *next = static_cast<R *>(j % 2 == 0 ? b.qa : b.qb);
        if (t.stages == 1) next = nullptr;
        naive_tab_stage<M, R, KAHAN><<<grid, block, 0, st>>>(y, b, arg, next, j, n, t);
        arg = next;
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
