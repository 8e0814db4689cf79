// naive.hip -- the standard implementation of an RK4 step (Sec. 2.2): one
// kernel per stage, each a full sweep over the chain whose results (the
// slope k_j and the next stage argument, Eq. 3-4) go through memory. Stage 4
// reads k1..k3 back and applies the final combination (Eq. 5) in place. It is
// the baseline the fused kernel is measured against, and it uses the same
// per-site operation order, so both give identical bits.
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
    // stage argument: y itself, then the ping-pong stage buffers
    const R *aq = STAGE == 1 ? yq : STAGE == 3 ? static_cast<const R *>(b.ybq) : static_cast<const R *>(b.yaq);
    const R *ap = STAGE == 1 ? yp : STAGE == 3 ? static_cast<const R *>(b.ybp) : static_cast<const R *>(b.yap);
    const StepConsts<R> c(dt);

    const R Qj = aq[i];
    const R Pj = ap[i];
    R F;
    if constexpr (coupling_range<M>() == 2) {
        const R b1l = ModelOps<M, R>::bond(Qj - aq[im]);
        const R b1r = ModelOps<M, R>::bond(aq[ip] - Qj);
        const R b2l = ModelOps<M, R>::bond(Qj - aq[wrap_index(i - 2, n)]);
        const R b2r = ModelOps<M, R>::bond(aq[wrap_index(i + 2, n)] - Qj);
        F = site_force2<M, R>(b1l, b1r, b2l, b2r, Qj);
    } else {
        const R bl = ModelOps<M, R>::bond(Qj - aq[im]);
        const R br = ModelOps<M, R>::bond(aq[ip] - Qj);
        F = site_force<M, R>(bl, br, Qj);
    }
    const R qj = yq[i];
    const R pj = yp[i];

    if constexpr (STAGE < 4) {
        R *kq = static_cast<R *>(STAGE == 1 ? b.k1q : STAGE == 2 ? b.k2q : b.k3q);
        R *kp = static_cast<R *>(STAGE == 1 ? b.k1p : STAGE == 2 ? b.k2p : b.k3p);
        R *nq = static_cast<R *>(STAGE == 2 ? b.ybq : b.yaq);
        R *np = static_cast<R *>(STAGE == 2 ? b.ybp : b.yap);
        const R a = STAGE == 3 ? c.h : c.hh;
        kq[i] = Pj;
        kp[i] = F;
        nq[i] = fma_r(a, Pj, qj);
        np[i] = fma_r(a, F, pj);
    } else {
        R accq = static_cast<const R *>(b.k1q)[i];
        R accp = static_cast<const R *>(b.k1p)[i];
        accq = fma_r(static_cast<R>(2), static_cast<const R *>(b.k2q)[i], accq);
        accp = fma_r(static_cast<R>(2), static_cast<const R *>(b.k2p)[i], accp);
        accq = fma_r(static_cast<R>(2), static_cast<const R *>(b.k3q)[i], accq);
        accp = fma_r(static_cast<R>(2), static_cast<const R *>(b.k3p)[i], accp);
        accq = accq + Pj;
        accp = accp + F;
        R *wq = static_cast<R *>(y.q);
        R *wp = static_cast<R *>(y.p);
        if constexpr (KAHAN) {
            R q1 = qj, p1 = pj;
            C *ycq = static_cast<C *>(y.cq), *ycp = static_cast<C *>(y.cp);
            C cq = ycq[i], cp = ycp[i];
            if constexpr (sizeof(C) == 8) {
                kahan_step(q1, cq, accq, c.h6d);
                kahan_step(p1, cp, accp, c.h6d);
            } else {
                kahan_step(q1, cq, accq, c.h6, c.h6lo);
                kahan_step(p1, cp, accp, c.h6, c.h6lo);
            }
            wq[i] = q1;
            wp[i] = p1;
            ycq[i] = cq;
            ycp[i] = cp;
        } else {
            wq[i] = fma_r(c.h6, accq, qj);
            wp[i] = fma_r(c.h6, accp, pj);
        }
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
