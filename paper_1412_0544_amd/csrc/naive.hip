// naive.hip -- the standard implementation of an RK4 step (Sec. 2.2): one
// kernel per stage, each a full sweep over the chain whose per-site results
// go through memory before the next stage reads them. It is the baseline the
// fused kernel is measured against, and it uses the same per-site operation
// order (site_update, site_final), so both give identical bits. What goes
// through memory: the stage argument (Q2 and Q4 in one array, Q3 in another),
// F1, the value site_update carries from stage 2 to 3 (F2; in the compensated
// FP32 forms also the increment it carries from stage 1 to 2) and the running
// sum F1 + F2 + F3.
#include "launch.hpp"
#include "rk4_device.hpp"

namespace chainrk4 {
namespace {

constexpr int kNaiveThreads = 256;

template <int M, class R, bool KAHAN, int STAGE, class C>
__global__ __launch_bounds__(kNaiveThreads) void naive_stage(StateRef y, NaiveBufs b, int64_t n,
                                                             double dt) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kNaiveThreads + threadIdx.x;
    if (i >= n) return;
    const int64_t im = (i == 0) ? n - 1 : i - 1;
    const int64_t ip = (i == n - 1) ? 0 : i + 1;
    const R *yq = static_cast<const R *>(y.q);
    const R *yp = static_cast<const R *>(y.p);
    R *Qa = static_cast<R *>(b.yaq);   // Q2, then Q4
    R *Qb = static_cast<R *>(b.ybq);   // Q3
    R *F1 = static_cast<R *>(b.k1p);
    R *F2 = static_cast<R *>(b.k2p);
    R *sum = static_cast<R *>(b.k2q);  // F1 + F2 (+ F3)
    // stage argument: q, Q2, Q3, Q4
    const R *arg = STAGE == 1 ? yq : STAGE == 3 ? Qb : Qa;
    const StepConsts<R, KAHAN> c(dt);

    const R Qj = arg[i];
    R F;
    if constexpr (coupling_range<M>() == 2) {
        const R b1l = ModelOps<M, R>::bond(Qj - arg[im]);
        const R b1r = ModelOps<M, R>::bond(arg[ip] - Qj);
        const R b2l = ModelOps<M, R>::bond(Qj - arg[wrap_index(i - 2, n)]);
        const R b2r = ModelOps<M, R>::bond(arg[wrap_index(i + 2, n)] - Qj);
        F = site_force2<M, R>(b1l, b1r, b2l, b2r, Qj);
    } else {
        const R bl = ModelOps<M, R>::bond(Qj - arg[im]);
        const R br = ModelOps<M, R>::bond(arg[ip] - Qj);
        F = site_force<M, R>(bl, br, Qj);
    }
    const R qj = yq[i];
    const R pj = yp[i];
    R Qo = Qj, X = 0, sj = 0, a = 0;
    if constexpr (STAGE == 1) {
        site_update<1>(F, Qj, Qo, X, qj, pj, sj, a, c);
        Qa[i] = Qo;
        F1[i] = a;
        if constexpr (KAHAN) F2[i] = X;
    } else if constexpr (STAGE == 2) {
        sj = F1[i];
        if constexpr (KAHAN) X = F2[i];
        site_update<2>(F, Qj, Qo, X, qj, pj, sj, a, c);
        Qb[i] = Qo;
        F2[i] = X;
        sum[i] = sj;
    } else if constexpr (STAGE == 3) {
        X = F2[i];
        sj = sum[i];
        site_update<3>(F, Qj, Qo, X, qj, pj, sj, a, c);
        Qa[i] = Qo;
        sum[i] = sj;
    } else {
        sj = sum[i];
        a = F1[i];
        site_update<4>(F, Qj, Qo, X, qj, pj, sj, a, c);
        R q1 = qj, p1 = pj;
        R *wq = static_cast<R *>(y.q);
        R *wp = static_cast<R *>(y.p);
        if constexpr (KAHAN) {
            C *ycq = static_cast<C *>(y.cq), *ycp = static_cast<C *>(y.cp);
            C cq = ycq[i], cp = ycp[i];
            site_final<R, true, C>(q1, p1, cq, cp, sj, a, c);
            ycq[i] = cq;
            ycp[i] = cp;
        } else {
            R unused = 0;
            site_final<R, false, R>(q1, p1, unused, unused, sj, a, c);
        }
        wq[i] = q1;
        wp[i] = p1;
    }
}

template <int M, class R, bool KAHAN, class C = float>
hipError_t naive_dispatch(StateRef y, const NaiveBufs &b, int64_t n, double dt, hipStream_t s) {
    const int64_t blocks = (n + kNaiveThreads - 1) / kNaiveThreads;
    if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(blocks)), block(kNaiveThreads);
    naive_stage<M, R, KAHAN, 1, C><<<grid, block, 0, s>>>(y, b, n, dt);
    naive_stage<M, R, KAHAN, 2, C><<<grid, block, 0, s>>>(y, b, n, dt);
    naive_stage<M, R, KAHAN, 3, C><<<grid, block, 0, s>>>(y, b, n, dt);
    naive_stage<M, R, KAHAN, 4, C><<<grid, block, 0, s>>>(y, b, n, dt);
    return hipGetLastError();
}

}  // namespace

template <int M>
hipError_t naive_dispatch_prec(int prec, StateRef y, const NaiveBufs &b, int64_t n, double dt,
                               hipStream_t s) {
    switch (prec) {
    case 0: return naive_dispatch<M, double, false>(y, b, n, dt, s);
    case 1: return naive_dispatch<M, float, true>(y, b, n, dt, s);
    case 2: return naive_dispatch<M, float, true, double>(y, b, n, dt, s);
    case 3: return naive_dispatch<M, float, false>(y, b, n, dt, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_naive_step(int model, int prec, StateRef y, const NaiveBufs &b, int64_t n,
                             double dt, hipStream_t s) {
    switch (model) {
    case kQuartic: return naive_dispatch_prec<kQuartic>(prec, y, b, n, dt, s);
    case kHarmonic: return naive_dispatch_prec<kHarmonic>(prec, y, b, n, dt, s);
    case kQuarticNNN: return naive_dispatch_prec<kQuarticNNN>(prec, y, b, n, dt, s);
    case kHarmonicNNN: return naive_dispatch_prec<kHarmonicNNN>(prec, y, b, n, dt, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace chainrk4
