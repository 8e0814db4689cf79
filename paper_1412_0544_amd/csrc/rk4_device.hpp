// rk4_device.hpp -- per-site arithmetic of the chain RK4 step, shared by every
// GPU kernel of the library so that all of them produce identical bits.
//
// The vector field is the homogeneous nearest-neighbour form of Sec. 2.1
// Eq. 2 written for a chain with coordinates q and momenta p:
//   dq_i/dt = p_i,  dp_i/dt = F_i = (phi(d_i) - phi(d_{i-1})) - U'(q_i),
//   d_i = q_{i+1} - q_i  (the bond to the right neighbour).
// quartic:  phi(d) = d^3, U'(q) = q + q^3 = q (1 + q^2)
// harmonic: phi(d) = d,   U'(q) = q
// Every bond term phi(d_i) is computed once and used by both sites it joins.
// The quartic on-site term is taken as q (1 + q^2) and subtracted from the
// bond difference by one fused multiply-add: 6 operations per site and stage
// (bond 3, 1 + q^2, difference, fma) instead of 7 for q + q^3 formed apart.
// The next-nearest-neighbour models (the generalisation of Sec. 5) add bonds
// to the second neighbours with the same phi:
//   F_i = ((phi(d_i) - phi(d_{i-1})) + (phi(e_i) - phi(e_{i-2}))) - U'(q_i),
//   e_i = q_{i+2} - q_i.
//
// One RK4 step (Sec. 2.2 Eq. 3-5, classical tableau) per site, h = dt:
//   stage j evaluates F at the stage argument (Q, P); k_j = (P, F)
//   acc = k1 + 2 k2 + 2 k3 + k4, accumulated in that order (the q part of
//   k1 is p, so its accumulation starts as fma(2, P2, p) in stage 2)
//   stage arguments: (Q, P) = (q, p) + a_j h k_j with a = (1/2, 1/2, 1)
//   final: y = y + (h/6) acc   (FP64: one fma; FP32: Kahan-compensated)
// Operation order is fixed here; kernels call these helpers only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chainrk4 {

enum Model : int { kQuartic = 0, kHarmonic = 1, kQuarticNNN = 3, kHarmonicNNN = 4 };

// Farthest neighbour the force reads.
template <int M>
constexpr int coupling_range() { return (M == kQuarticNNN || M == kHarmonicNNN) ? 2 : 1; }

// Fused multiply-add in the working precision (one rounding).
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int M, class R>
struct ModelOps;

template <class R>
struct ModelOps<kQuartic, R> {
    __device__ __forceinline__ static R bond(R d) { return (d * d) * d; }
    // t - U'(q) with U'(q) = q (1 + q^2): one rounding for 1 + q^2, one for
    // the fused product and difference
    __device__ __forceinline__ static R force(R t, R q) {
        return fma_r(-fma_r(q, q, static_cast<R>(1)), q, t);
    }
    // energy density of the site and its right bond, in FP64
    __device__ __forceinline__ static double energy(double q, double p, double d) {
        double q2 = q * q, d2 = d * d;
        return 0.5 * (p * p) + 0.5 * q2 + 0.25 * (q2 * q2) + 0.25 * (d2 * d2);
    }
};

template <class R>
struct ModelOps<kHarmonic, R> {
    __device__ __forceinline__ static R bond(R d) { return d; }
    __device__ __forceinline__ static R force(R t, R q) { return t - q; }
    __device__ __forceinline__ static double energy(double q, double p, double d) {
        return 0.5 * (p * p) + 0.5 * (q * q) + 0.5 * (d * d);
    }
};

// The NNN models reuse the bond and on-site terms of their NN model.
template <class R>
struct ModelOps<kQuarticNNN, R> : ModelOps<kQuartic, R> {
    // energy density of the site and its two right bonds, in FP64
    __device__ __forceinline__ static double energy2(double q, double p, double d, double e) {
        double q2 = q * q, d2 = d * d, e2 = e * e;
        return 0.5 * (p * p) + 0.5 * q2 + 0.25 * (q2 * q2) + 0.25 * (d2 * d2) + 0.25 * (e2 * e2);
    }
};

template <class R>
struct ModelOps<kHarmonicNNN, R> : ModelOps<kHarmonic, R> {
    __device__ __forceinline__ static double energy2(double q, double p, double d, double e) {
        return 0.5 * (p * p) + 0.5 * (q * q) + 0.5 * (d * d) + 0.5 * (e * e);
    }
};

// Force on a site from its left bond term, right bond term and coordinate.
template <int M, class R>
__device__ __forceinline__ R site_force(R bl, R br, R q) {
    return ModelOps<M, R>::force(br - bl, q);
}

// NNN force from the four bond terms that meet at the site:
// b1l = phi(q_i - q_{i-1}), b1r = phi(q_{i+1} - q_i),
// b2l = phi(q_i - q_{i-2}), b2r = phi(q_{i+2} - q_i).
template <int M, class R>
__device__ __forceinline__ R site_force2(R b1l, R b1r, R b2l, R b2r, R q) {
    return ModelOps<M, R>::force((b1r - b1l) + (b2r - b2l), q);
}

// Step constants in the working precision. The products of two step factors
// (hh2, hhh, h26) are formed in FP64 and rounded once. SPLIT selects the
// stage arguments of the compensated FP32 forms (site_update).
template <class R, bool SPLIT = false>
struct StepConsts {
    R h, hh, h6;
    R hh2;       // (h/2)^2
    R hhh;       // h * h/2
    R h26;       // h^2/6
    R hlo;       // dt - h: with h it gives dt to about twice R's precision
    R h6lo;      // dt/6 - h6, the same for dt/6
    R h26lo;     // dt^2/6 - h26, the same for dt^2/6
    double hd, h6d, h26d;  // dt, dt/6, dt^2/6 in FP64 (FP64 carries)
    __device__ __forceinline__ explicit StepConsts(double dt)
        : h(static_cast<R>(dt)),
          hh(static_cast<R>(0.5) * static_cast<R>(dt)),
          h6(static_cast<R>(dt / 6.0)),
          hh2(static_cast<R>((0.5 * dt) * (0.5 * dt))),
          hhh(static_cast<R>(dt * (0.5 * dt))),
          h26(static_cast<R>(dt * dt / 6.0)),
          hlo(static_cast<R>(dt - static_cast<double>(static_cast<R>(dt)))),
          h6lo(static_cast<R>(dt / 6.0 - static_cast<double>(static_cast<R>(dt / 6.0)))),
          h26lo(static_cast<R>(dt * dt / 6.0 - static_cast<double>(static_cast<R>(dt * dt / 6.0)))),
          hd(dt),
          h6d(dt / 6.0),
          h26d(dt * dt / 6.0) {}
};

// Kahan-compensated update of y with carry c (the true value is y - c): the
// caller forms v = increment - c; kahan_finish adds it to y and keeps the new
// rounding error in c.
__device__ __forceinline__ void kahan_finish(float &y, float &c, float v) {
    const float t = y + v;
    c = (t - y) - v;
    y = t;
}

// The same with an FP64 carry: the increment and the carry stay in FP64, only
// the running value y is FP32 (its rounding error goes to the carry; t - y of
// two FP32 values is exact in FP64).
__device__ __forceinline__ void kahan_finish(float &y, double &c, double v) {
    const float t = static_cast<float>(static_cast<double>(y) + v);
    c = (static_cast<double>(t) - static_cast<double>(y)) - v;
    y = t;
}

// y += (hi + lo) acc, compensated. The step factor comes in two FP32 parts
// (hi + lo = h to about 48 bits), so the increment carries no systematic FP32
// rounding of h: a factor rounded once to FP32 scales every step's increment
// by the same (1 + eps), a first-order error that the carry cannot undo. Two
// fused multiply-adds form v = (hi + lo) acc - c with one final rounding, the
// same instruction count as a product and a difference.
__device__ __forceinline__ void kahan_step(float &y, float &c, float acc, float hi, float lo) {
    kahan_finish(y, c, __builtin_fmaf(hi, acc, __builtin_fmaf(lo, acc, -c)));
}

// The same with an FP64 carry: the increment h acc is formed in FP64.
__device__ __forceinline__ void kahan_step(float &y, double &c, float acc, double h) {
    kahan_finish(y, c, h * static_cast<double>(acc) - c);
}

// ---------------------------------------------------------------------------
// Wavefront neighbour exchange (wave64, DPP). from_right(x): lane i receives
// lane i+1's x; lane 63 receives 0. from_left(x): lane i receives lane i-1's
// x; lane 0 receives 0. The kernels only use those edge lanes' results inside
// the recomputed halo (or replace them from LDS), so the zeros never reach
// output; filling with zero lets the move write a fresh register instead of
// first copying the source.
// ---------------------------------------------------------------------------
constexpr int kDppWaveShl1 = 0x130;  // wave_shl:1
constexpr int kDppWaveShr1 = 0x138;  // wave_shr:1

template <int Ctrl>
__device__ __forceinline__ int dpp32(int x) {
    return __builtin_amdgcn_mov_dpp(x, Ctrl, 0xF, 0xF, true);
}

template <int Ctrl>
__device__ __forceinline__ double dpp(double x) {
    int lo = __double2loint(x), hi = __double2hiint(x);
    lo = dpp32<Ctrl>(lo);
    hi = dpp32<Ctrl>(hi);
    return __hiloint2double(hi, lo);
}

template <int Ctrl>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(dpp32<Ctrl>(__float_as_int(x)));
}

template <class R>
__device__ __forceinline__ R from_right(R x) { return dpp<kDppWaveShl1>(x); }
template <class R>
__device__ __forceinline__ R from_left(R x) { return dpp<kDppWaveShr1>(x); }

// ---------------------------------------------------------------------------
// The per-site part of stage STAGE once the force F_STAGE at the stage
// argument Q_STAGE is known.
//
// For dq/dt = p, dp/dt = F(q) the q slopes of RK4 (Eq. 3-5) are the p stage
// values P_j = p + a_j h F_{j-1}, so every q quantity follows from p and the
// forces (exact algebra; only the rounding differs from the stage-by-stage
// form):
//   Q2 = q + (h/2) p,   Q3 = Q2 + (h/2)^2 F1,   Q4 = q + h p + h (h/2) F2,
//   q' = q + h p + (h^2/6)(F1 + F2 + F3),
//   p' = p + (h/6)(F1 + 2 F2 + 2 F3 + F4),  F1 + 2F2 + 2F3 + F4 = 2(F1 + F2 + F3) + F4 - F1.
// The P_j are never formed: 11 operations per site and step besides the four
// forces, against 14 for the stage-by-stage form. Per site, between stages:
//   Qo  the stage argument, overwritten with the next one (Qj: its old value)
//   X   F2 (stage 2 to 3)
//   s   F1 + F2 + F3 (stages 1 to 3)
//   a   F1 (stages 1 to 4); after stage 4, F1 + 2F2 + 2F3 + F4
//
// The compensated FP32 forms (SPLIT) take the step factor of the stage
// arguments in two parts as well: where dt is not an FP32 number, R(dt)
// differs from dt by up to 3e-8 relative, and stage arguments formed with it
// perturb the method's second-order condition (sum b_j c_j = 1/2) by that
// much. On an oscillation of frequency w that is an energy gain of about
// 3e-8 (w h)^2 per step, the same in every step: at dt = 0.01 over 10^4 steps
// as large as RK4's own dissipation. The two parts only help if the small one
// is added before the increment meets q (q + lo p rounds back to q), so the
// increment is formed apart, u = hi p + lo p, and added to q last:
//   Q2 = q + u/2,  X = u + h (h/2) F2 (stage 2 to 3),  Q4 = q + X,
// two operations more per site and step (X carries u from stage 1 to 2).
// ---------------------------------------------------------------------------
template <int STAGE, class R, bool SPLIT>
__device__ __forceinline__ void site_update(R F, R Qj, R &Qo, R &X, R qj, R pj, R &s, R &a,
                                            const StepConsts<R, SPLIT> &c) {
    if (STAGE == 1) {
        a = F;
        s = F;
        if constexpr (SPLIT) {
            X = fma_r(c.h, pj, c.hlo * pj);
            Qo = fma_r(static_cast<R>(0.5), X, qj);
        } else {
            Qo = fma_r(c.hh, pj, qj);
        }
    } else if (STAGE == 2) {
        Qo = fma_r(c.hh2, s, Qj);
        if constexpr (SPLIT)
            X = fma_r(c.hhh, F, X);
        else
            X = F;
        s = s + F;
    } else if (STAGE == 3) {
        if constexpr (SPLIT)
            Qo = qj + X;
        else
            Qo = fma_r(c.hhh, X, fma_r(c.h, pj, qj));
        s = s + F;
    } else {
        a = fma_r(static_cast<R>(2), s, F) - a;
    }
}

// The end of the step for one site: q' = q + h p + (h^2/6) s, p' = p + (h/6) a
// (s, a as left by stage 4). FP64 and plain FP32 round each operation. The
// compensated FP32 forms keep the rounding of each update in the carry (FP32,
// or FP64 with the increment formed in FP64), and take every step factor of
// the increment in two FP32 parts (hi + lo): a factor rounded once to FP32
// scales the same term of every step alike, an error the carry cannot undo.
// For h that is a first-order error; for h^2/6 it is an energy drift of order
// eps h^2 per step, which a split removes too (one more fused multiply-add).
template <class R, bool KAHAN, class C, bool SPLIT>
__device__ __forceinline__ void site_final(R &q, R &p, C &cq, C &cp, R s, R a,
                                           const StepConsts<R, SPLIT> &c) {
    if constexpr (!KAHAN) {
        q = fma_r(c.h26, s, fma_r(c.h, p, q));
        p = fma_r(c.h6, a, p);
    } else if constexpr (sizeof(C) == 8) {
        kahan_finish(q, cq, fma_r(c.h26d, static_cast<double>(s),
                                  fma_r(c.hd, static_cast<double>(p), -cq)));
        kahan_step(p, cp, a, c.h6d);
    } else {
        kahan_finish(q, cq, fma_r(c.h, p, fma_r(c.hlo, p, fma_r(c.h26, s, fma_r(c.h26lo, s, -cq)))));
        kahan_step(p, cp, a, c.h6, c.h6lo);
    }
}

// ---------------------------------------------------------------------------
// One RK4 stage over the S consecutive sites a lane holds.
//   Q       stage argument (in), overwritten with the next stage argument
//   q, p    state at the start of the step
//   X, s, a per-site values carried between stages (site_update)
//   bl0     bond term left of site 0; brS bond term right of site S-1
// Stage 1 reads its argument from q (Q is an output only).
// ---------------------------------------------------------------------------
template <int M, int S, int STAGE, class R, bool SPLIT>
__device__ __forceinline__ void stage_sites(R (&Q)[S], R (&X)[S], R (&q)[S], R (&p)[S],
                                            R (&s)[S], R (&a)[S], R bl0, R brS,
                                            const StepConsts<R, SPLIT> &c) {
    R bl = bl0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const R Qj = (STAGE == 1) ? q[j] : Q[j];
        R br;
        if (j + 1 < S) {
            const R Qn = (STAGE == 1) ? q[j + 1] : Q[j + 1];
            br = ModelOps<M, R>::bond(Qn - Qj);
        } else {
            br = brS;
        }
        const R F = site_force<M, R>(bl, br, Qj);
        bl = br;
        site_update<STAGE>(F, Qj, Q[j], X[j], q[j], p[j], s[j], a[j], c);
    }
}

// One RK4 stage over S consecutive sites of a next-nearest-neighbour chain
// (S >= 2). The edge bond terms come from the neighbour lanes:
//   b1l0 = phi(Q_0 - Q_{-1}),  b2lm2 = phi(Q_0 - Q_{-2}),  b2lm1 = phi(Q_1 - Q_{-1}),
//   b1rS = phi(Q_S - Q_{S-1}), b2rS2 = phi(Q_S - Q_{S-2}), b2rS1 = phi(Q_{S+1} - Q_{S-1}).
template <int M, int S, int STAGE, class R, bool SPLIT>
__device__ __forceinline__ void stage_sites_nnn(R (&Q)[S], R (&X)[S], R (&q)[S], R (&p)[S],
                                                R (&s)[S], R (&a)[S], R b1l0, R b2lm2, R b2lm1,
                                                R b1rS, R b2rS2, R b2rS1,
                                                const StepConsts<R, SPLIT> &c) {
    static_assert(S >= 2, "a lane holds at least two sites");
    R b1l = b1l0, b2l_lo = b2lm2, b2l_hi = b2lm1;  // phi of bonds (j-1, j), (j-2, j), (j-1, j+1)
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const R Qj = (STAGE == 1) ? q[j] : Q[j];
        R b1r, b2r;
        if (j + 1 < S) b1r = ModelOps<M, R>::bond(((STAGE == 1) ? q[j + 1] : Q[j + 1]) - Qj);
        else b1r = b1rS;
        if (j + 2 < S) b2r = ModelOps<M, R>::bond(((STAGE == 1) ? q[j + 2] : Q[j + 2]) - Qj);
        else b2r = (j + 2 == S) ? b2rS2 : b2rS1;
        const R F = site_force2<M, R>(b1l, b1r, b2l_lo, b2r, Qj);
        b1l = b1r;
        b2l_lo = b2l_hi;
        b2l_hi = b2r;
        site_update<STAGE>(F, Qj, Q[j], X[j], q[j], p[j], s[j], a[j], c);
    }
}

// The end of the step (Eq. 5) for the S sites of a lane: without
// compensation, and with the carries of the compensated FP32 forms.
template <int S, class R, bool SPLIT>
__device__ __forceinline__ void final_update(R (&q)[S], R (&p)[S], const R (&s)[S],
                                             const R (&a)[S], const StepConsts<R, SPLIT> &c) {
#pragma unroll
    for (int j = 0; j < S; ++j) {
        R unused = 0;
        site_final<R, false, R>(q[j], p[j], unused, unused, s[j], a[j], c);
    }
}

template <int S, class C, bool SPLIT>
__device__ __forceinline__ void final_update_kahan(float (&q)[S], float (&p)[S], C (&cq)[S],
                                                   C (&cp)[S], const float (&s)[S],
                                                   const float (&a)[S],
                                                   const StepConsts<float, SPLIT> &c) {
#pragma unroll
    for (int j = 0; j < S; ++j) site_final<float, true, C>(q[j], p[j], cq[j], cp[j], s[j], a[j], c);
}

// Same arithmetic for one site held alone (resident kernel).
template <int M, int STAGE, class R, bool SPLIT>
__device__ __forceinline__ void stage_one(R Qm, R Qj, R Qp, R qj, R pj, R &X, R &s, R &a, R &Qn,
                                          const StepConsts<R, SPLIT> &c) {
    const R bl = ModelOps<M, R>::bond(Qj - Qm);
    const R br = ModelOps<M, R>::bond(Qp - Qj);
    const R F = site_force<M, R>(bl, br, Qj);
    site_update<STAGE>(F, Qj, Qn, X, qj, pj, s, a, c);
}

// ---------------------------------------------------------------------------
// Roessler chain (Sec. 3.1 Eq. 6-7), FP64, three coordinates per site:
//   dx/dt = (d_i - d_{i-1}) - (y + z),  d_i = x_{i+1} - x_i
//   dy/dt = x + a y,   dz/dt = b + z (x - c),   a = 0.2, b = 1, c = 9.
// ---------------------------------------------------------------------------
struct Roessler {
    static constexpr double a = 0.2, b = 1.0, c = 9.0;
    __device__ __forceinline__ static void rhs(double bl, double br, double X, double Y, double Z,
                                               double &kx, double &ky, double &kz) {
        kx = (br - bl) - (Y + Z);
        ky = fma_r(a, Y, X);
        kz = fma_r(Z, X - c, b);
    }
};

// One RK4 stage of the Roessler chain over S consecutive sites (same
// structure as stage_sites; only x couples to the neighbours).
template <int S, int STAGE>
__device__ __forceinline__ void roessler_stage_sites(double (&X)[S], double (&Y)[S], double (&Z)[S],
                                                     double (&x)[S], double (&y)[S], double (&z)[S],
                                                     double (&ax)[S], double (&ay)[S],
                                                     double (&az)[S], double bl0, double brS,
                                                     const StepConsts<double> &c) {
    double bl = bl0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const double Xj = (STAGE == 1) ? x[j] : X[j];
        const double Yj = (STAGE == 1) ? y[j] : Y[j];
        const double Zj = (STAGE == 1) ? z[j] : Z[j];
        double br;
        if (j + 1 < S)
            br = ((STAGE == 1) ? x[j + 1] : X[j + 1]) - Xj;
        else
            br = brS;
        double kx, ky, kz;
        Roessler::rhs(bl, br, Xj, Yj, Zj, kx, ky, kz);
        bl = br;
        if (STAGE == 1) {
            ax[j] = kx; ay[j] = ky; az[j] = kz;
            X[j] = fma_r(c.hh, kx, x[j]); Y[j] = fma_r(c.hh, ky, y[j]); Z[j] = fma_r(c.hh, kz, z[j]);
        } else if (STAGE == 2) {
            ax[j] = fma_r(2.0, kx, ax[j]); ay[j] = fma_r(2.0, ky, ay[j]); az[j] = fma_r(2.0, kz, az[j]);
            X[j] = fma_r(c.hh, kx, x[j]); Y[j] = fma_r(c.hh, ky, y[j]); Z[j] = fma_r(c.hh, kz, z[j]);
        } else if (STAGE == 3) {
            ax[j] = fma_r(2.0, kx, ax[j]); ay[j] = fma_r(2.0, ky, ay[j]); az[j] = fma_r(2.0, kz, az[j]);
            X[j] = fma_r(c.h, kx, x[j]); Y[j] = fma_r(c.h, ky, y[j]); Z[j] = fma_r(c.h, kz, z[j]);
        } else {
            ax[j] = ax[j] + kx; ay[j] = ay[j] + ky; az[j] = az[j] + kz;
            x[j] = fma_r(c.h6, ax[j], x[j]);
            y[j] = fma_r(c.h6, ay[j], y[j]);
            z[j] = fma_r(c.h6, az[j], z[j]);
        }
    }
}

// Ring index of an unwrapped site index (any sign, any multiple of n).
__device__ __forceinline__ int64_t wrap_index(int64_t i, int64_t n) {
    if (i >= 0 && i < n) return i;
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

}  // namespace chainrk4
