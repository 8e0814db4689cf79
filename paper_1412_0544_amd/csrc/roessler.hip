// roessler.hip -- the paper's own workload, the Roessler chain (Sec. 3.1),
// with the same two implementations as the Hamiltonian chains: the fused,
// temporally blocked cluster pass (Sec. 2.3; the overlap of s sites per side
// carried over `ksteps` steps) and the standard one-kernel-per-stage sweep
// (Sec. 2.2). Only x couples to the neighbours, so only x crosses lanes.
#include "cluster.hpp"

namespace chainrk4 {
namespace {

constexpr int roessler_block_threads(int W) { return W == 1 ? kFusedThreads : 64 * W; }

// Edge x values of every lane of a block, double-buffered by stage parity.
template <int NL>
struct LaneEdges {
    double first[2][NL], last[2][NL];
};

// One stage of the Roessler chain for the S sites of this lane. Only x
// crosses lanes. A one-wavefront cluster moves the edge values by DPP. A
// cluster of several wavefronts has every lane publish its first and last x
// in LDS and read its neighbours' after one barrier: no lane-dependent
// branches, which holds the kernel to 92 VGPRs (5 wavefronts per SIMD)
// instead of 117 with DPP plus two LDS slots per wavefront. The bond term
// x_{i} - x_{i-1} across two lanes is the same operation on the same values
// in both lanes, so the result does not depend on the route.
template <int S, int STAGE, int W, int NL>
__device__ __forceinline__ void roessler_lane_stage(double (&X)[S], double (&Y)[S], double (&Z)[S],
                                                    double (&x)[S], double (&y)[S], double (&z)[S],
                                                    double (&ax)[S], double (&ay)[S],
                                                    double (&az)[S], const StepConsts<double> &c,
                                                    LaneEdges<NL> *edges, int gl, int parity) {
    const double first = (STAGE == 1) ? x[0] : X[0];
    const double last = (STAGE == 1) ? x[S - 1] : X[S - 1];
    double brS, bl0;
    if constexpr (W > 1) {
        edges->first[parity][gl] = first;
        edges->last[parity][gl] = last;
        __syncthreads();
        // the cluster's outermost lanes read a clamped or foreign value: their
        // sites lie in the recomputed halo
        const double right = edges->first[parity][gl + 1 < NL ? gl + 1 : gl];
        const double left = edges->last[parity][gl > 0 ? gl - 1 : gl];
        brS = right - last;
        bl0 = first - left;
    } else {
        brS = from_right(first) - last;
        bl0 = from_left(brS);
    }
    roessler_stage_sites<S, STAGE>(X, Y, Z, x, y, z, ax, ay, az, bl0, brS, c);
}

template <int S>
__device__ __forceinline__ void load3(double (&x)[S], double (&y)[S], double (&z)[S],
                                      const StateRef &in, int64_t n, int64_t s0, bool contiguous) {
    const double *xi = static_cast<const double *>(in.q);
    const double *yi = static_cast<const double *>(in.p);
    if (contiguous) {
        load_contig<double, S>(x, xi + s0);
        load_contig<double, S>(y, yi + s0);
        load_contig<double, S>(z, in.z + s0);
    } else {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int64_t i = wrap_index(s0 + j, n);
            x[j] = xi[i];
            y[j] = yi[i];
            z[j] = in.z[i];
        }
    }
}

template <int S, int W>
__global__ __launch_bounds__(roessler_block_threads(W)) void roessler_fused_kernel(FusedPass a) {
    constexpr int WPB = roessler_block_threads(W) / 64;
    constexpr int CPB = WPB / W;
    constexpr int E = 64 * S * W;
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int wic = wib % W;
    const int64_t cluster = static_cast<int64_t>(blockIdx.x) * CPB + wib / W;
    constexpr int NL = W > 1 ? WPB * 64 : 1;
    __shared__ LaneEdges<NL> edges;
    if (cluster >= a.waves) return;  // W = 1 only (a W > 1 grid has no extra blocks)
    const int64_t e0 = cluster * a.tile - a.halo;
    const int lo = (wic * 64 + lane) * S;
    const int64_t s0 = e0 + lo;
    double x[S], y[S], z[S];
    load3<S>(x, y, z, a.in, a.n, s0, e0 >= 0 && e0 + E <= a.n);
    const StepConsts<double> c(a.dt);
    double X[S], Y[S], Z[S], ax[S], ay[S], az[S];
    for (int k = 0; k < a.ksteps; ++k) {
        roessler_lane_stage<S, 1, W, NL>(X, Y, Z, x, y, z, ax, ay, az, c, &edges, wib * 64 + lane, 0);
        roessler_lane_stage<S, 2, W, NL>(X, Y, Z, x, y, z, ax, ay, az, c, &edges, wib * 64 + lane, 1);
        roessler_lane_stage<S, 3, W, NL>(X, Y, Z, x, y, z, ax, ay, az, c, &edges, wib * 64 + lane, 0);
        roessler_lane_stage<S, 4, W, NL>(X, Y, Z, x, y, z, ax, ay, az, c, &edges, wib * 64 + lane, 1);
    }
    double *xo = static_cast<double *>(a.out.q);
    double *yo = static_cast<double *>(a.out.p);
    const int64_t keep_hi = a.halo + a.tile;
    if (lo >= a.halo && lo + S <= keep_hi && s0 + S <= a.n) {
        store_contig<double, S>(xo + s0, x);
        store_contig<double, S>(yo + s0, y);
        store_contig<double, S>(a.out.z + s0, z);
    } else {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int64_t g = s0 + j;
            if (lo + j >= a.halo && lo + j < keep_hi && g < a.n) {
                xo[g] = x[j];
                yo[g] = y[j];
                a.out.z[g] = z[j];
            }
        }
    }
}

constexpr int kNaiveThreads = 256;

// The standard implementation for the Roessler chain: stage j reads its
// argument and the state, writes the slope k_j and the next argument; stage 4
// combines k1..k4 (Eq. 5) in place.
template <int STAGE>
__global__ __launch_bounds__(kNaiveThreads) void roessler_naive_stage(StateRef y, NaiveBufs b,
                                                                      int64_t n, double dt) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kNaiveThreads + threadIdx.x;
    if (i >= n) return;
    const int64_t im = (i == 0) ? n - 1 : i - 1;
    const int64_t ip = (i == n - 1) ? 0 : i + 1;
    const double *yx = static_cast<const double *>(y.q);
    const double *yy = static_cast<const double *>(y.p);
    const double *ax = STAGE == 1 ? yx : STAGE == 3 ? static_cast<const double *>(b.ybq)
                                                    : static_cast<const double *>(b.yaq);
    const double *ay = STAGE == 1 ? yy : STAGE == 3 ? static_cast<const double *>(b.ybp)
                                                    : static_cast<const double *>(b.yap);
    const double *az = STAGE == 1 ? y.z : STAGE == 3 ? b.ybz : b.yaz;
    const StepConsts<double> c(dt);
    const double Xj = ax[i];
    const double bl = Xj - ax[im];
    const double br = ax[ip] - Xj;
    double kx, ky, kz;
    Roessler::rhs(bl, br, Xj, ay[i], az[i], kx, ky, kz);
    const double xj = yx[i], yj = yy[i], zj = y.z[i];
    if constexpr (STAGE < 4) {
        double *kxo = static_cast<double *>(STAGE == 1 ? b.k1q : STAGE == 2 ? b.k2q : b.k3q);
        double *kyo = static_cast<double *>(STAGE == 1 ? b.k1p : STAGE == 2 ? b.k2p : b.k3p);
        double *kzo = STAGE == 1 ? b.k1z : STAGE == 2 ? b.k2z : b.k3z;
        double *nx = static_cast<double *>(STAGE == 2 ? b.ybq : b.yaq);
        double *ny = static_cast<double *>(STAGE == 2 ? b.ybp : b.yap);
        double *nz = STAGE == 2 ? b.ybz : b.yaz;
        const double s = STAGE == 3 ? c.h : c.hh;
        kxo[i] = kx;
        kyo[i] = ky;
        kzo[i] = kz;
        nx[i] = fma_r(s, kx, xj);
        ny[i] = fma_r(s, ky, yj);
        nz[i] = fma_r(s, kz, zj);
    } else {
        const double *k1x = static_cast<const double *>(b.k1q), *k2x = static_cast<const double *>(b.k2q),
                     *k3x = static_cast<const double *>(b.k3q);
        const double *k1y = static_cast<const double *>(b.k1p), *k2y = static_cast<const double *>(b.k2p),
                     *k3y = static_cast<const double *>(b.k3p);
        double sx = k1x[i], sy = k1y[i], sz = b.k1z[i];
        sx = fma_r(2.0, k2x[i], sx); sy = fma_r(2.0, k2y[i], sy); sz = fma_r(2.0, b.k2z[i], sz);
        sx = fma_r(2.0, k3x[i], sx); sy = fma_r(2.0, k3y[i], sy); sz = fma_r(2.0, b.k3z[i], sz);
        sx = sx + kx; sy = sy + ky; sz = sz + kz;
        static_cast<double *>(y.q)[i] = fma_r(c.h6, sx, xj);
        static_cast<double *>(y.p)[i] = fma_r(c.h6, sy, yj);
        y.z[i] = fma_r(c.h6, sz, zj);
    }
}

template <int S, int W>
hipError_t roessler_launch_one(const FusedPass &a, hipStream_t st) {
    constexpr int T = roessler_block_threads(W);
    constexpr int cpb = T / 64 / W;
    const int64_t blocks64 = (a.waves + cpb - 1) / cpb;
    if (blocks64 <= 0 || blocks64 > 0x7fffffff) return hipErrorInvalidValue;
    roessler_fused_kernel<S, W><<<dim3(static_cast<unsigned>(blocks64)), dim3(T), 0, st>>>(a);
    return hipGetLastError();
}

template <int S>
hipError_t roessler_dispatch_w(int w, const FusedPass &a, hipStream_t st) {
    switch (w) {
    case 1: return roessler_launch_one<S, 1>(a, st);
    case 2: return roessler_launch_one<S, 2>(a, st);
    case 4: return roessler_launch_one<S, 4>(a, st);
    case 8: return roessler_launch_one<S, 8>(a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fused_roessler(int s, int w, const FusedPass &a, hipStream_t st) {
    switch (s) {
    case 4: return roessler_dispatch_w<4>(w, a, st);
    case 8: return roessler_dispatch_w<8>(w, a, st);
    case 16: return roessler_dispatch_w<16>(w, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_naive_roessler_step(StateRef y, const NaiveBufs &b, int64_t n, double dt,
                                      hipStream_t st) {
    const int64_t blocks = (n + kNaiveThreads - 1) / kNaiveThreads;
    if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(blocks)), block(kNaiveThreads);
    roessler_naive_stage<1><<<grid, block, 0, st>>>(y, b, n, dt);
    roessler_naive_stage<2><<<grid, block, 0, st>>>(y, b, n, dt);
    roessler_naive_stage<3><<<grid, block, 0, st>>>(y, b, n, dt);
    roessler_naive_stage<4><<<grid, block, 0, st>>>(y, b, n, dt);
    return hipGetLastError();
}

}  // namespace chainrk4
