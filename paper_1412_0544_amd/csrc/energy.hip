// energy.hip -- total energy of a chain in FP64, and a zero-fill kernel.
//
// H = sum_i e_i with e_i the kinetic and on-site energy of site i plus the
// potential of its bond to site i+1 (and to site i+2 with second-neighbour
// bonds): the Hamiltonian whose gradient is the force of the model. For the
// FP32 state with compensated update each coordinate enters as
// (hi - carry), in FP64. Each block sums a fixed,
// strided subset of sites and reduces it with a fixed tree; one finishing
// block sums the partials the same way. The grid depends only on n, so the
// result is the same bits on every call.
#include "launch.hpp"
#include "rk4_device.hpp"

namespace chainrk4 {
namespace {

template <class R, bool KAHAN, class C>
__device__ __forceinline__ void coords(const StateRef &y, int64_t i, double &q, double &p) {
    const R *yq = static_cast<const R *>(y.q);
    const R *yp = static_cast<const R *>(y.p);
    if constexpr (KAHAN) {
        q = static_cast<double>(yq[i]) - static_cast<double>(static_cast<const C *>(y.cq)[i]);
        p = static_cast<double>(yp[i]) - static_cast<double>(static_cast<const C *>(y.cp)[i]);
    } else {
        q = static_cast<double>(yq[i]);
        p = static_cast<double>(yp[i]);
    }
}

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double s[kEnergyThreads];
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
#pragma unroll
    for (int w = kEnergyThreads / 2; w > 0; w >>= 1) {
        if (t < w) s[t] = s[t] + s[t + w];
        __syncthreads();
    }
    return s[0];
}

// Energy of site i: its kinetic and on-site terms and the bond(s) to the right.
template <int M, class R, bool KAHAN, class C>
__device__ __forceinline__ double site_energy(const StateRef &y, int64_t n, int64_t i) {
    const int64_t ip = (i == n - 1) ? 0 : i + 1;
    double q, p, qn, pn;
    coords<R, KAHAN, C>(y, i, q, p);
    coords<R, KAHAN, C>(y, ip, qn, pn);
    if constexpr (coupling_range<M>() == 2) {
        double qnn, pnn;
        coords<R, KAHAN, C>(y, wrap_index(i + 2, n), qnn, pnn);
        return ModelOps<M, double>::energy2(q, p, qn - q, qnn - q);
    } else {
        return ModelOps<M, double>::energy(q, p, qn - q);
    }
}

// Each thread sums the sites i0, i0 + stride, i0 + 2*stride, ... in that
// order. The loads of four consecutive terms are issued together (more bytes
// in flight per wavefront), and the terms are still added one by one in index
// order, so the sum is the same bits as a plain strided loop.
template <int M, class R, bool KAHAN, class C>
__global__ __launch_bounds__(kEnergyThreads) void energy_partial(StateRef y, int64_t n,
                                                                 double *partials) {
    constexpr int U = 4;
    double acc = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kEnergyThreads;
    int64_t i = static_cast<int64_t>(blockIdx.x) * kEnergyThreads + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        double e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) e[u] = site_energy<M, R, KAHAN, C>(y, n, i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) acc += e[u];
    }
    for (; i < n; i += stride) acc += site_energy<M, R, KAHAN, C>(y, n, i);
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kEnergyThreads) void energy_finish(const double *partials, int nb,
                                                                double *result) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += kEnergyThreads) acc += partials[b];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) result[0] = s;
}

__global__ void fill_zero_kernel(uint32_t *p, size_t words) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < words; i += stride)
        p[i] = 0u;
}

template <int M, class R, bool KAHAN, class C = float>
hipError_t energy_dispatch(StateRef y, int64_t n, double *partials, double *result, hipStream_t s) {
    const int nb = energy_blocks(n);
    energy_partial<M, R, KAHAN, C><<<nb, kEnergyThreads, 0, s>>>(y, n, partials);
    energy_finish<<<1, kEnergyThreads, 0, s>>>(partials, nb, result);
    return hipGetLastError();
}

}  // namespace

int energy_blocks(int64_t n) {
    int64_t nb = (n + 4 * kEnergyThreads - 1) / (4 * kEnergyThreads);
    if (nb < 1) nb = 1;
    if (nb > kEnergyMaxBlocks) nb = kEnergyMaxBlocks;
    return static_cast<int>(nb);
}

template <int M>
hipError_t energy_dispatch_prec(int prec, StateRef y, int64_t n, double *partials, double *result,
                                hipStream_t s) {
    switch (prec) {
    case 0: return energy_dispatch<M, double, false>(y, n, partials, result, s);
    case 1: return energy_dispatch<M, float, true>(y, n, partials, result, s);
    case 2: return energy_dispatch<M, float, true, double>(y, n, partials, result, s);
    case 3: return energy_dispatch<M, float, false>(y, n, partials, result, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_energy(int model, int prec, StateRef y, int64_t n, double *partials,
                         double *result, hipStream_t s) {
    switch (model) {
    case kQuartic: return energy_dispatch_prec<kQuartic>(prec, y, n, partials, result, s);
    case kHarmonic: return energy_dispatch_prec<kHarmonic>(prec, y, n, partials, result, s);
    case kQuarticNNN: return energy_dispatch_prec<kQuarticNNN>(prec, y, n, partials, result, s);
    case kHarmonicNNN: return energy_dispatch_prec<kHarmonicNNN>(prec, y, n, partials, result, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    const size_t words = bytes / 4;
    size_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    fill_zero_kernel<<<static_cast<unsigned>(blocks), 256, 0, s>>>(static_cast<uint32_t *>(ptr), words);
    return hipGetLastError();
}

}  // namespace chainrk4
