// roessler.hip -- the paper's own workload, the Roessler chain (Sec. 3.1),
// with the same two implementations as the Hamiltonian chains: the fused,
// temporally blocked cluster pass (Sec. 2.3; the overlap of s sites per side
// carried over `ksteps` steps) and the standard one-kernel-per-stage sweep
// (Sec. 2.2). Only x couples to the neighbours, so only x crosses lanes.
#include <atomic>

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
    steps_by_progress(0, a.ksteps, a.balance ? a.ksteps : 0, [&] {
        roessler_lane_stage<S, 1, W, NL>(X, Y, Z, x, y, z, ax, ay, az, c, &edges, wib * 64 + lane, 0);
        roessler_lane_stage<S, 2, W, NL>(X, Y, Z, x, y, z, ax, ay, az, c, &edges, wib * 64 + lane, 1);
        roessler_lane_stage<S, 3, W, NL>(X, Y, Z, x, y, z, ax, ay, az, c, &edges, wib * 64 + lane, 0);
        roessler_lane_stage<S, 4, W, NL>(X, Y, Z, x, y, z, ax, ay, az, c, &edges, wib * 64 + lane, 1);
    });
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

// A whole step call of the Roessler chain with every cluster held in
// registers by one workgroup (see ExchangeRun). Each pass is the fused
// kernel's cluster pass: the same per-site arithmetic and an overlap of at
// least reach * steps sites per side (Sec. 2.3), so the kept sites are the
// exact RK4 result and the bits equal the fused path's. Between passes only
// the kept sites a neighbour reads move through memory, instead of every
// site of the chain being stored and loaded again: the first `zone` kept
// sites (the left neighbour's right halo) and the last `halo` (the right
// neighbour's left halo). They are written with device-coherent stores and
// read with device-coherent loads, since the neighbour may run on another
// XCD; a cluster marks its pass done only after its stores completed.
//
// Exchange buffers by pass parity: pass j writes into back (j even) or
// front (j odd), and the call has an even number of passes, so the last pass
// stores into the caller's buffers. A buffer is written again two passes
// later, by which time both readers have moved on (a cluster finishing pass
// j + 2 has waited for its neighbours to finish pass j + 1, which they start
// only after reading their pass-j halo). The first writes into front come
// from pass 1, after the neighbours have finished pass 0 and so have read
// their initial state.
template <int S, int W>
__global__ __launch_bounds__(64 * W) void roessler_exchange_kernel(ExchangeRun a) {
    constexpr int E = 64 * S * W;
    constexpr int NL = W > 1 ? 64 * W : 1;
    __shared__ LaneEdges<NL> edges;
    // each wavefront's staging area for the edge sites it hands on
    __shared__ __align__(16) double stage[W * 64 * S];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int gl = wib * 64 + lane;
    const int g = blockIdx.x;
    const int G = a.clusters;
    const int64_t start = 4 * (static_cast<int64_t>(g) * a.uq + (g < a.ur ? g : a.ur));
    const int64_t keep = (g == G - 1) ? a.n - start : 4 * (a.uq + (g < a.ur ? 1 : 0));
    const int64_t e0 = start - a.halo;
    const int lo = gl * S;
    const int64_t s0 = e0 + lo;
    double x[S], y[S], z[S];
    load3<S>(x, y, z, a.front, a.n, s0, e0 >= 0 && e0 + E <= a.n);
    const StepConsts<double> c(a.dt);
    double X[S], Y[S], Z[S], ax[S], ay[S], az[S];
    const int64_t base = a.steps / a.passes, extra = a.steps % a.passes;
    const int left = g == 0 ? G - 1 : g - 1, right = g == G - 1 ? 0 : g + 1;
    // issue priority by progress over the whole call (not per pass: a
    // cluster that enters its next pass early must not take precedence over
    // an unrelated one on the same SIMD still finishing the previous pass)
    int64_t done = 0;
    for (int pass = 0;; ++pass) {
        const int64_t k = base + (pass < extra ? 1 : 0);
        steps_by_progress(done, k, a.steps, [&] {
            roessler_lane_stage<S, 1, W, NL>(X, Y, Z, x, y, z, ax, ay, az, c, &edges, gl, 0);
            roessler_lane_stage<S, 2, W, NL>(X, Y, Z, x, y, z, ax, ay, az, c, &edges, gl, 1);
            roessler_lane_stage<S, 3, W, NL>(X, Y, Z, x, y, z, ax, ay, az, c, &edges, gl, 0);
            roessler_lane_stage<S, 4, W, NL>(X, Y, Z, x, y, z, ax, ay, az, c, &edges, gl, 1);
        });
        done += k;
        if (pass + 1 == a.passes) break;
        const StateRef ex = (pass & 1) ? a.front : a.back;
        double *xe = static_cast<double *>(ex.q);
        double *ye = static_cast<double *>(ex.p);
        double *ze = ex.z;
        // Positions again from the lane id, hidden from the compiler, and in
        // 32 bits inside the cluster: nothing of this is kept live through
        // the step loop (which holds the kernel at 5 wavefronts per SIMD).
        int lane_x = gl;
        asm volatile("" : "+v"(lane_x));
        const int lx = lane_x * S;
        const int h = static_cast<int>(a.halo), kp = static_cast<int>(keep);
        const int zn = static_cast<int>(a.zone);
        const int64_t sx = e0 + lx;
        // The kept sites the neighbours read: the first `zone` (the left
        // neighbour's right halo) and the last `halo`. Kept sites never wrap
        // (site e0 + pos is start + pos - halo < n); the buffer resource spans
        // the cluster's window from its origin e0, which may lie before the
        // array, and only kept sites, inside it, are written. Staged through
        // LDS, each store instruction covers consecutive 16-byte pieces.
        auto handed = [h, kp, zn](int pos) {
            return pos >= h && pos < h + kp && (pos < h + zn || pos >= kp);
        };
        constexpr int bytes = E * static_cast<int>(sizeof(double));
        const int wv = lane_x >> 6, ln = lane_x & 63;  // wavefront in the block, lane
        double *st = stage + wv * 64 * S;
        const int wlo = wv * 64 * S;                    // the wavefront's first local site
        store_staged<double, S>(st, x, xe + e0, bytes, ln, wlo, handed);
        store_staged<double, S>(st, y, ye + e0, bytes, ln, wlo, handed);
        store_staged<double, S>(st, z, ze + e0, bytes, ln, wlo, handed);
        drain_memory();
        __syncthreads();
        if (threadIdx.x == 0) {
            store_flag(a.flags + g, a.base + pass + 1);
            wait_flags(a.flags + left, a.flags + g, a.flags + right, a.base + pass + 1, a.error,
                       a.spin_limit);
        }
        __syncthreads();
        // halo sites lie within one cluster of the kept ones and n exceeds a
        // cluster (checked by the host), so one wrap suffices
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int local = lx + j;
            if (local < h || local >= h + kp) {
                int64_t i = sx + j;
                i = i < 0 ? i + a.n : (i >= a.n ? i - a.n : i);
                x[j] = load_coherent(xe + i);
                y[j] = load_coherent(ye + i);
                z[j] = load_coherent(ze + i);
            }
        }
    }
    // the last pass is odd: its kept sites go to the caller's buffers
    int lane_s = gl;
    asm volatile("" : "+v"(lane_s));
    const int lo_s = lane_s * S;
    const int64_t s0_s = e0 + lo_s;
    double *xo = static_cast<double *>(a.front.q);
    double *yo = static_cast<double *>(a.front.p);
    if (lo_s >= a.halo && lo_s + S <= a.halo + keep) {
        store_contig<double, S>(xo + s0_s, x);
        store_contig<double, S>(yo + s0_s, y);
        store_contig<double, S>(a.front.z + s0_s, z);
    } else {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (lo_s + j >= a.halo && lo_s + j < a.halo + keep) {
                xo[s0_s + j] = x[j];
                yo[s0_s + j] = y[j];
                a.front.z[s0_s + j] = z[j];
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
    FusedPass b = a;
    b.balance = blocks64 <= resident_blocks<roessler_fused_kernel<S, W>>(T) ? 1 : 0;
    roessler_fused_kernel<S, W><<<dim3(static_cast<unsigned>(blocks64)), dim3(T), 0, st>>>(b);
    return hipGetLastError();
}

template <int S, int W>
hipError_t exchange_launch_one(const ExchangeRun &a, hipStream_t st) {
    if (a.clusters < 3 || a.passes < 2 || (a.passes & 1)) return hipErrorInvalidValue;
    roessler_exchange_kernel<S, W><<<dim3(static_cast<unsigned>(a.clusters)), dim3(64 * W), 0, st>>>(a);
    return hipGetLastError();
}

template <int S, int W>
int exchange_capacity_one() {
    return resident_blocks<roessler_exchange_kernel<S, W>>(64 * W);
}

template <int S>
hipError_t exchange_dispatch_w(int w, const ExchangeRun &a, hipStream_t st) {
    switch (w) {
    case 1: return exchange_launch_one<S, 1>(a, st);
    case 2: return exchange_launch_one<S, 2>(a, st);
    case 4: return exchange_launch_one<S, 4>(a, st);
    case 8: return exchange_launch_one<S, 8>(a, st);
    default: return hipErrorInvalidValue;
    }
}

template <int S>
int exchange_capacity_w(int w) {
    switch (w) {
    case 1: return exchange_capacity_one<S, 1>();
    case 2: return exchange_capacity_one<S, 2>();
    case 4: return exchange_capacity_one<S, 4>();
    case 8: return exchange_capacity_one<S, 8>();
    default: return 0;
    }
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
    case 6: return roessler_dispatch_w<6>(w, a, st);
    case 8: return roessler_dispatch_w<8>(w, a, st);
    case 16: return roessler_dispatch_w<16>(w, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_exchange_roessler(int s, int w, const ExchangeRun &a, hipStream_t st) {
    switch (s) {
    case 4: return exchange_dispatch_w<4>(w, a, st);
    case 6: return exchange_dispatch_w<6>(w, a, st);
    case 8: return exchange_dispatch_w<8>(w, a, st);
    default: return hipErrorInvalidValue;
    }
}

int exchange_capacity_roessler(int s, int w) {
    switch (s) {
    case 4: return exchange_capacity_w<4>(w);
    case 6: return exchange_capacity_w<6>(w);
    case 8: return exchange_capacity_w<8>(w);
    default: return 0;
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
