// chain_rk4.cpp -- host side of the C ABI declared in include/chain_rk4.h:
// argument validation, workspace layout, the pass plan of a step call, graph
// capture, and the energy read-back.
#include "chain_rk4.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "handle.hpp"
#include "launch.hpp"

using namespace chainrk4;

namespace chainrk4 {

thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(CHAIN_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t elem_bytes(int prec) { return prec == CHAIN_FP64 ? sizeof(double) : sizeof(float); }
bool has_carries(int prec) { return prec == CHAIN_FP32_KAHAN || prec == CHAIN_FP32_KAHAN64; }
size_t carry_bytes(int prec) { return prec == CHAIN_FP32_KAHAN64 ? sizeof(double) : sizeof(float); }

bool is_gfx950(int dev) {
    // 0 unknown, 1 yes, 2 no; handles on different threads may ask at once
    static std::atomic<int> cached[64];
    if (dev < 0 || dev >= 64) return false;
    int v = cached[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
        v = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
        cached[dev].store(v, std::memory_order_relaxed);
    }
    return v == 1;
}

}  // namespace chainrk4

namespace {

constexpr size_t kAlign = 256;
size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Defaults when the descriptor leaves the tile shape to the library.
constexpr int kDefaultSitesFp64 = 8;
constexpr int kDefaultSitesFp32 = 16;
constexpr int kDefaultWaves = 4;

// Cluster shape of the quartic and harmonic chains by chain length: the
// fastest (S, W, k) of sweeps over S = 2..16, W = 1..8, k = 4..32 and
// N = 2^10..2^26 on MI355X (the granularity study of Sec. 2.3 and 3.2.1).
// Short chains want many small one-wavefront clusters (no barriers, every
// CU busy, few instructions per wavefront and step); long ones want few halo
// sites per kept site. FP64, with the 6-operation force: a chain that fills
// the chip about once is fastest where its sites per SIMD come closest to
// a whole number of wavefronts (6 sites per lane at 2^18-2^19 and in
// four-wavefront clusters at 2^21, 10-27% over the shapes before). Up to
// 2^14 sites the chip is far from full and a call's time is its passes'
// latency, so passes of 28 steps (halo 56 of each 128-site cluster) beat
// 16: a 1000-step call on 1024 sites takes 0.26 instead of 0.32 ms. Long
// chains keep four-wavefront clusters of 8 sites per lane at depth 32:
// one-wavefront clusters of 16 (214 registers, 2 wavefronts per SIMD, no
// barriers) at depth 24 ran 1000-step jobs at N = 2^24 1.6-1.8% faster on
// two boxes, but a 50-step call then takes 4 passes instead of 2 (N = 2^26:
// 6.4 against 7.8e11 site-updates/s), and at depth 32 they were level
// (+2.4% and -0.8%).
struct ShapeRow {
    int64_t max_n;
    int sites, waves, depth;
};
constexpr ShapeRow kShapeFp64[] = {{int64_t(1) << 14, 2, 1, 28},
                                   {int64_t(1) << 16, 2, 1, 16},
                                   {int64_t(1) << 17, 4, 1, 32},
                                   {int64_t(1) << 19, 6, 1, 32},
                                   {int64_t(1) << 20, 8, 1, 32},
                                   {int64_t(1) << 21, 6, 4, 32},
                                   {INT64_MAX, 8, 4, 32}};
// FP32 state: passes of 28 steps up to 2^14 sites and one-wavefront clusters
// of 4 sites per lane at 2^17 as for FP64 (1000-step calls 12-18% and 10-12%
// faster than 2 sites per lane at depth 16); multi-wavefront clusters from
// 2^18 sites on, where the all-lane
// LDS exchange leaves room for more sites per lane. Plain FP32 takes 16 sites
// per lane on long chains; the compensated forms stay at 8, where their split
// stage arguments keep 95 registers (5 wavefronts per SIMD; at 16 they took
// 169, or spilled under a 128 bound, and ran 5 to 7% slower).
constexpr ShapeRow kShapeFp32[] = {{int64_t(1) << 14, 2, 1, 28},
                                   {int64_t(1) << 16, 2, 1, 16},
                                   {int64_t(1) << 17, 4, 1, 32},
                                   {int64_t(1) << 19, 2, 4, 32},
                                   {int64_t(1) << 21, 4, 4, 32},
                                   {int64_t(1) << 23, 8, 4, 32},
                                   {INT64_MAX, 16, 4, 32}};
constexpr ShapeRow kShapeFp32Kahan[] = {{int64_t(1) << 14, 2, 1, 28},
                                        {int64_t(1) << 16, 2, 1, 16},
                                        {int64_t(1) << 17, 4, 1, 32},
                                        {int64_t(1) << 19, 2, 4, 32},
                                        {int64_t(1) << 21, 4, 4, 32},
                                        {INT64_MAX, 8, 4, 32}};

template <size_t K>
ShapeRow row_for(const ShapeRow (&rows)[K], int64_t n) {
    for (size_t i = 0; i < K; ++i)
        if (n <= rows[i].max_n) return rows[i];
    return rows[K - 1];
}

ShapeRow shape_for(int prec, int64_t n) {
    if (prec == CHAIN_FP64) return row_for(kShapeFp64, n);
    if (prec == CHAIN_FP32) return row_for(kShapeFp32, n);
    return row_for(kShapeFp32Kahan, n);
}
// Roessler: nine S-site register arrays per lane instead of six (92
// registers at 4 sites per lane, 128 at 6, 166 at 8). Fused passes, from
// sweeps over S, W, k: chains up to 2^21 sites take 4 sites per lane at
// depth 25 (halo 100; at N = 2^20 the chain fills the chip about once, so
// each pass pays its load and store with little overlap, and fewer, deeper
// passes measured faster: 3.7 against 3.4e11 SU/s for 50-step calls at depth
// 16); longer chains 8 sites per lane at depth 25 (5.50 against 4.88e11 SU/s
// for 4 sites per lane at depth 16, N = 2^24).
constexpr int kDefaultWavesRoessler = 4;
constexpr int kRoesslerDepth = 25;
// Shorter Roessler chains (fused passes, library shape): one-wavefront
// clusters while the chip is far from full; a 1000-step call on 2^10..2^14
// sites took 0.52 instead of 0.86 ms with 4 sites per lane at depth 25 in
// one wavefront, 0.61 against 0.86 ms at 2^16 at depth 16, and 0.99 against
// 1.14 ms at 2^18 with 8 sites per lane; from 2^19 on the rows above hold.
constexpr ShapeRow kShapeRoessler[] = {{int64_t(1) << 14, 4, 1, 25},
                                       {int64_t(1) << 16, 4, 1, 16},
                                       {int64_t(1) << 18, 8, 1, 25},
                                       {int64_t(1) << 21, 4, 4, 25},
                                       {INT64_MAX, 8, 4, 25}};
// FP64 chains with second-neighbour bonds (reach 4 per step): the same for
// short chains (1000-step calls at 2^10..2^14 sites 0.46-0.49 against
// 2.05 ms with the long-chain shape, 0.64 against 2.07 at 2^16, 1.06
// against 2.09 at 2^18, 2.85 against 3.59 at 2^20); from 2^21 on four
// wavefronts of 8 sites per lane at depth 16 (the best of a sweep at 2^22).
constexpr ShapeRow kShapeNnnFp64[] = {{int64_t(1) << 14, 2, 1, 14},
                                      {int64_t(1) << 16, 2, 1, 8},
                                      {int64_t(1) << 18, 4, 1, 16},
                                      {int64_t(1) << 20, 8, 1, 16},
                                      {INT64_MAX, 8, 4, 16}};
// The plain and compensated FP32 forms of those chains (one table for both:
// their timings rank the shapes alike): 1000-step calls at 2^10..2^14 sites
// 0.44 against 2.92 ms (compensated) with the long-chain shape, 0.59 against
// 3.05 at 2^16, 1.12 against 3.07 at 2^18, 2.25 against 3.24 at 2^20 in four
// wavefronts of 4 sites per lane, 6.32 against 7.26 at 2^22 with 8 per lane;
// longer chains keep 16 sites per lane.
constexpr ShapeRow kShapeNnnFp32[] = {{int64_t(1) << 14, 2, 1, 14},
                                      {int64_t(1) << 16, 2, 1, 8},
                                      {int64_t(1) << 18, 4, 1, 16},
                                      {int64_t(1) << 20, 4, 4, 16},
                                      {int64_t(1) << 22, 8, 4, 16},
                                      {INT64_MAX, 16, 4, 16}};
// Tableau passes up to 2^18 sites: one wavefront of 4 sites per lane at the
// default depth (FP64: 1000 steps of 2^10..2^16 sites 0.49 against 1.37 ms
// for the 3/8-rule tableau, 0.68 against 1.62 ms for Dormand-Prince 5; at
// 2^18 0.78 against 1.40 and 1.22 against 2.00 ms; compensated FP32: 0.64
// against 1.56 and 0.92 against 1.53 ms, at 2^18 0.90 against 1.58 and 1.36
// against 1.56). Compensated FP32 up to 2^20: four wavefronts of 4 sites per
// lane (2.01 against 2.32 ms for the 3/8 rule; Dormand-Prince 5 has them).
constexpr int64_t kTableauShortSites = int64_t(1) << 18;
constexpr int64_t kTableauMidSitesFp32 = int64_t(1) << 20;
// FP64 four-stage tableaus up to 2^20 sites: one wavefront of 8 sites per
// lane (2.05 against 2.54 ms for 1000 steps of the 3/8 rule at 2^20).
constexpr int64_t kTableauMidSitesFp64 = int64_t(1) << 20;
constexpr int64_t kRoesslerShortSites = int64_t(1) << 21;
constexpr int kRoesslerShortSitesPerLane = 4;
constexpr int kRoesslerLongSitesPerLane = 8;
// CHAIN_FLAG_EXCHANGE: between passes only the edge sites move, in place of
// the whole chain's store and reload, so shallower passes (less overlap)
// pay: depth 13 (halo 52) measured 4.84 against 4.60e11 SU/s for depth 25
// at N = 2^20 in 50-step calls. Every cluster stays resident for the call,
// so the chip's share of each SIMD sets the pace: 2^20 sites are 1024 per
// SIMD, which 4 sites per lane hold in 5 wavefronts of 256 (1280 lane-sites
// per SIMD with the halo), and 6 sites per lane in 3 of 384 (1152; 735
// clusters, about 3 per CU): 5.21 against 4.96e11 SU/s at depth 13.
constexpr int kExchangeDepthRoessler = 13;
constexpr int kExchangeSitesRoessler = 6;
// Default depth: as many steps as a halo of 64 sites per side covers (32 for
// the NN chains, 16 for the NNN and Roessler chains; the fastest depth of a
// sweep over S, W, k at N = 2^24 and N = 2^20).
constexpr int kDefaultHalo = 64;
constexpr int kMaxDepth = 32;

bool valid_sites(int s) { return s == 2 || s == 4 || s == 8 || s == 16; }
bool valid_waves(int w) { return w == 1 || w == 2 || w == 4 || w == 8; }

int check_desc(const chain_rk4_desc *d) {
    if (!d) return fail(CHAIN_EINVAL, "descriptor is NULL");
    if (d->n < 1) return fail(CHAIN_EINVAL, "n must be >= 1 (got %lld)", (long long)d->n);
    if (d->n > (int64_t(1) << 40)) return fail(CHAIN_EINVAL, "n too large");
    if (d->model != CHAIN_QUARTIC && d->model != CHAIN_HARMONIC && d->model != CHAIN_ROESSLER &&
        d->model != CHAIN_QUARTIC_NNN && d->model != CHAIN_HARMONIC_NNN)
        return fail(CHAIN_EINVAL, "unknown model %d", d->model);
    if (d->prec != CHAIN_FP64 && d->prec != CHAIN_FP32_KAHAN && d->prec != CHAIN_FP32_KAHAN64 &&
        d->prec != CHAIN_FP32)
        return fail(CHAIN_EINVAL, "unknown precision %d", d->prec);
    if (d->model == CHAIN_ROESSLER && d->prec != CHAIN_FP64)
        return fail(CHAIN_EINVAL, "the Roessler chain runs in FP64 only");
    if (!std::isfinite(d->dt)) return fail(CHAIN_EINVAL, "dt must be finite");
    if (d->method != CHAIN_FUSED && d->method != CHAIN_NAIVE)
        return fail(CHAIN_EINVAL, "unknown method %d", d->method);
    if (d->model == CHAIN_ROESSLER) {
        // six sites per lane (128 registers, 4 wavefronts per SIMD) is built
        // for the Roessler kernels only
        if (d->sites_per_lane != 0 && d->sites_per_lane != 6 &&
            (d->sites_per_lane == 2 || !valid_sites(d->sites_per_lane)))
            return fail(CHAIN_EINVAL, "the Roessler kernel takes sites_per_lane 0, 4, 6, 8 or 16 (got %d)",
                        d->sites_per_lane);
    } else if (d->sites_per_lane == 6) {
        // six sites per lane: the classical RK4 pass of the FP64 nearest-
        // neighbour chains (96 registers, 5 wavefronts per SIMD)
        if ((d->model != CHAIN_QUARTIC && d->model != CHAIN_HARMONIC) || d->prec != CHAIN_FP64 ||
            d->scheme != CHAIN_SCHEME_RK4 || d->method != CHAIN_FUSED)
            return fail(CHAIN_EINVAL, "sites_per_lane 6 takes the fused classical RK4 of the FP64 "
                                      "quartic and harmonic chains (and the Roessler chain)");
    } else if (d->sites_per_lane != 0 && !valid_sites(d->sites_per_lane)) {
        return fail(CHAIN_EINVAL, "sites_per_lane must be 0, 2, 4, 6, 8 or 16 (got %d)", d->sites_per_lane);
    }
    if (d->kdepth < 0 || d->kdepth > kMaxDepth)
        return fail(CHAIN_EINVAL, "kdepth must be in 0..%d (got %d)", kMaxDepth, d->kdepth);
    if (d->waves_per_cluster != 0 && !valid_waves(d->waves_per_cluster))
        return fail(CHAIN_EINVAL, "waves_per_cluster must be 0, 1, 2, 4 or 8 (got %d)",
                    d->waves_per_cluster);
    if (d->scheme != CHAIN_SCHEME_RK4 && d->scheme != CHAIN_SCHEME_TABLEAU)
        return fail(CHAIN_EINVAL, "unknown scheme %d", d->scheme);
    if (d->scheme == CHAIN_SCHEME_TABLEAU) {
        if (d->model == CHAIN_ROESSLER)
            return fail(CHAIN_EINVAL, "a tableau method is not available for the Roessler chain");
        if (d->prec == CHAIN_FP32_KAHAN64 || d->prec == CHAIN_FP32)
            return fail(CHAIN_EINVAL, "tableau methods take CHAIN_FP64 or CHAIN_FP32_KAHAN");
    }
    if (d->flags &
        ~(CHAIN_FLAG_GRAPH | CHAIN_FLAG_NO_RESIDENT | CHAIN_FLAG_RESIDENT | CHAIN_FLAG_EXCHANGE))
        return fail(CHAIN_EINVAL, "unknown flags 0x%x", d->flags);
    if ((d->flags & CHAIN_FLAG_EXCHANGE) &&
        (d->model != CHAIN_ROESSLER || d->method != CHAIN_FUSED || (d->flags & CHAIN_FLAG_RESIDENT)))
        return fail(CHAIN_EINVAL, "CHAIN_FLAG_EXCHANGE takes the Roessler chain on the fused method");
    if ((d->flags & CHAIN_FLAG_EXCHANGE) && d->sites_per_lane > 8)
        return fail(CHAIN_EINVAL, "CHAIN_FLAG_EXCHANGE takes sites_per_lane 4, 6 or 8");
    if (d->flags & CHAIN_FLAG_RESIDENT) {
        if (d->flags & CHAIN_FLAG_NO_RESIDENT)
            return fail(CHAIN_EINVAL, "CHAIN_FLAG_RESIDENT and CHAIN_FLAG_NO_RESIDENT exclude each other");
        if (d->n > kResidentMaxSites)
            return fail(CHAIN_EINVAL, "a resident ring holds at most %d sites", kResidentMaxSites);
        if ((d->model != CHAIN_QUARTIC && d->model != CHAIN_HARMONIC) ||
            d->scheme != CHAIN_SCHEME_RK4 || d->method != CHAIN_FUSED)
            return fail(CHAIN_EINVAL, "resident rings run the classical RK4 of the quartic and "
                                      "harmonic chains on the fused path only");
        if (d->prec == CHAIN_FP32_KAHAN64 || d->prec == CHAIN_FP32)
            return fail(CHAIN_EINVAL, "resident rings take CHAIN_FP64 or CHAIN_FP32_KAHAN");
    }
    return CHAIN_OK;
}

// Polls (each with a short sleep) before a cluster of an exchange run gives
// up waiting for its neighbours: seconds, far beyond any pass.
constexpr int kExchangeSpinLimit = 1 << 22;

// The cluster plan of a descriptor (defined below, after the reach helpers).
Plan make_plan(const chain_rk4_desc *d, int64_t reach_override = 0, int stages = 4);

// Arrays of N values the per-stage method of the Hamiltonian chains keeps.
constexpr int kNaiveArraysHamiltonian = 5;

// Workspace regions, in order. Unused regions have size 0.
struct Layout {
    size_t back_q, back_p, back_z;    // fused: back buffer of the ping-pong
    size_t cq, cp, back_cq, back_cp;  // FP32 state: carries (front and back)
    size_t naive[10];                 // naive: k1..k3 and two stage arguments (Roessler;
                                      // the Hamiltonian chains take the first 5)
    size_t naive_z[5];                // naive, Roessler: the same for z
    size_t naive_tab[(kMaxStages - 1) + 2];  // naive tableau: forces, two arguments
    size_t partials, result;          // energy
    size_t xflags, xerror;            // CHAIN_FLAG_EXCHANGE: pass counters, timeout word
    size_t total;
};

Layout layout(const chain_rk4_desc *d) {
    Layout L{};
    const size_t n = static_cast<size_t>(d->n);
    const size_t arr = round_up(n * elem_bytes(d->prec));
    const size_t carr = round_up(n * carry_bytes(d->prec));
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += bytes;
        return o;
    };
    const bool kahan = has_carries(d->prec);
    const bool three = d->model == CHAIN_ROESSLER;
    if (d->method == CHAIN_FUSED) {
        L.back_q = take(arr);
        L.back_p = take(arr);
        if (three) L.back_z = take(arr);
    }
    if (kahan) {
        L.cq = take(carr);
        L.cp = take(carr);
        if (d->method == CHAIN_FUSED) {
            L.back_cq = take(carr);
            L.back_cp = take(carr);
        }
    }
    if (d->method == CHAIN_NAIVE && d->scheme == CHAIN_SCHEME_TABLEAU) {
        for (size_t &o : L.naive_tab) o = take(arr);
    } else if (d->method == CHAIN_NAIVE) {
        for (int i = 0; i < (three ? 10 : kNaiveArraysHamiltonian); ++i) L.naive[i] = take(arr);
        if (three)
            for (int i = 0; i < 5; ++i) L.naive_z[i] = take(arr);
    }
    L.partials = take(round_up(kEnergyMaxBlocks * sizeof(double)));
    L.result = take(kAlign);
    if (d->flags & CHAIN_FLAG_EXCHANGE) {
        const Plan P = make_plan(d);
        L.xflags = take(round_up(static_cast<size_t>(P.waves) * sizeof(int32_t)));
        L.xerror = take(kAlign);
    }
    L.total = off;
    return L;
}


// Sites per side that one step's wrong edge values travel into a cluster
// (Sec. 2.3: one per stage and coupling range for a field that couples every
// coordinate, as the Roessler chain's x; for dq/dt = p with coupling only in
// dp/dt the stage arguments of stages 1 and 2 move q locally, so the front
// advances one site per two stages).
int64_t step_reach(int model) {
    switch (model) {
    case CHAIN_QUARTIC:
    case CHAIN_HARMONIC: return 2;
    case CHAIN_QUARTIC_NNN:
    case CHAIN_HARMONIC_NNN: return 4;
    default: return 4;  // CHAIN_ROESSLER
    }
}

// Reach of one step of an explicit tableau for dq/dt = p, dp/dt = F(q) with
// F reaching `range` sites: the stage argument Q_j combines momenta P_m,
// P_j combines forces F(Q_m); a zero coefficient adds nothing.
int64_t tableau_reach_of(const TabArgs &t, int64_t range) {
    int64_t rq[kMaxStages] = {0}, rp[kMaxStages] = {0};
    for (int j = 1; j < t.stages; ++j)
        for (int m = 0; m < j; ++m)
            if (t.a[j][m] != 0.0) {
                rq[j] = std::max(rq[j], rp[m]);
                rp[j] = std::max(rp[j], rq[m] + range);
            }
    int64_t r = 0;
    for (int m = 0; m < t.stages; ++m)
        if (t.b[m] != 0.0) r = std::max(r, std::max(rp[m], rq[m] + range));
    return r;
}

int64_t model_range(int model) {
    return (model == CHAIN_QUARTIC_NNN || model == CHAIN_HARMONIC_NNN) ? 2 : 1;
}

// Sites in one 16-byte vector of the state arrays (the FP64-carry form's
// carries need 2, its FP32 coordinates 4). A lane loads and stores its S
// consecutive sites with 16-byte vector accesses when its cluster does not
// wrap, so the cluster's first site must sit on such a boundary: the halo is
// rounded up to a whole number of vectors. A wider overlap than the reach
// needs keeps the kept sites exact (Sec. 2.3), so the bits do not change.
int64_t vector_sites(int prec) { return prec == CHAIN_FP64 ? 2 : 4; }

// Cluster shape of the tableau kernel (see launch_tableau).
bool tableau_shape_ok(int stages, int sites, int waves) {
    if (waves != 1 && waves != 4) return false;
    return stages <= 4 ? (sites == 4 || sites == 8) : sites == 4;
}

// Tableau kernel: 8 sites per lane up to 4 stages, 4 beyond (the registers
// hold every stage's slope); the fastest in a sweep over S, W, k at N = 2^24.
int default_sites_tableau(int stages) { return stages <= 4 ? 8 : 4; }

Plan make_plan(const chain_rk4_desc *d, int64_t reach_override, int stages) {
    Plan P;
    if (d->method != CHAIN_FUSED) return P;
    const bool roessler = d->model == CHAIN_ROESSLER;
    const bool nn = d->model == CHAIN_QUARTIC || d->model == CHAIN_HARMONIC;
    const bool tab = d->scheme == CHAIN_SCHEME_TABLEAU;
    if (d->flags & CHAIN_FLAG_RESIDENT) {  // validated: NN model, classical RK4, short ring
        P.resident = true;
        return P;
    }
    const ShapeRow row = shape_for(d->prec, d->n);
    // library shapes by chain length (when neither S nor W is given)
    const bool free_shape = !d->sites_per_lane && !d->waves_per_cluster;
    const bool roe_table = roessler && !(d->flags & CHAIN_FLAG_EXCHANGE) && free_shape;
    const bool nnn_table = (d->model == CHAIN_QUARTIC_NNN || d->model == CHAIN_HARMONIC_NNN) &&
                           (d->prec == CHAIN_FP64 || d->prec == CHAIN_FP32 ||
                            d->prec == CHAIN_FP32_KAHAN) &&
                           !tab && free_shape;
    const bool tab_tuned = tab && free_shape && (d->prec == CHAIN_FP64 || d->prec == CHAIN_FP32_KAHAN);
    const bool tab_short = tab_tuned && d->n <= kTableauShortSites;
    const bool tab_one = tab_short || (tab_tuned && d->prec == CHAIN_FP64 && stages == 4 &&
                                       d->n <= kTableauMidSitesFp64);
    const bool tab_four = tab_short || (tab_tuned && d->prec == CHAIN_FP32_KAHAN &&
                                        d->n <= kTableauMidSitesFp32);
    const ShapeRow rrow = row_for(kShapeRoessler, d->n);
    const ShapeRow nrow = d->prec == CHAIN_FP64 ? row_for(kShapeNnnFp64, d->n)
                                                 : row_for(kShapeNnnFp32, d->n);
    P.sites = d->sites_per_lane ? d->sites_per_lane
              : roessler && (d->flags & CHAIN_FLAG_EXCHANGE)
                  ? kExchangeSitesRoessler
              : roe_table       ? rrow.sites
              : nnn_table       ? nrow.sites
              : roessler        ? (d->n <= kRoesslerShortSites ? kRoesslerShortSitesPerLane
                                                               : kRoesslerLongSitesPerLane)
              : tab_four        ? 4
              : tab             ? default_sites_tableau(stages)
              : nn              ? row.sites
              : (d->prec == CHAIN_FP64 ? kDefaultSitesFp64 : kDefaultSitesFp32);
    P.waves_per_cluster = d->waves_per_cluster ? d->waves_per_cluster
                          : roe_table            ? rrow.waves
                          : nnn_table            ? nrow.waves
                          : tab_one              ? 1
                          : roessler             ? kDefaultWavesRoessler
                          : nn && !tab           ? row.waves
                                                 : kDefaultWaves;
    const int64_t reach = reach_override > 0 ? reach_override : step_reach(d->model);
    const bool table_shape = nn && !tab && !d->sites_per_lane && !d->waves_per_cluster;
    P.depth = d->kdepth      ? d->kdepth
              : table_shape ? row.depth
              : roessler && (d->flags & CHAIN_FLAG_EXCHANGE)
                  ? kExchangeDepthRoessler
              : roe_table ? rrow.depth
              : nnn_table ? nrow.depth
              : roessler ? kRoesslerDepth
                  : static_cast<int>(std::min<int64_t>(
                        kMaxDepth, std::max<int64_t>(1, kDefaultHalo / reach)));
    const int64_t E = 64 * static_cast<int64_t>(P.sites) * P.waves_per_cluster;
    const int64_t V = vector_sites(d->prec);
    auto halo_of = [&](int depth) { return (reach * depth + V - 1) / V * V; };
    // the kept part of a cluster must stay positive: E > 2*halo. E is a
    // multiple of 128 sites, so the tile, and with it every cluster origin
    // cluster*tile - halo, stays a whole number of vectors.
    while (E <= 2 * halo_of(P.depth) && P.depth > 1) --P.depth;
    P.halo = halo_of(P.depth);
    P.tile = E - 2 * P.halo;
    P.waves = (d->n + P.tile - 1) / P.tile;
    if ((d->flags & CHAIN_FLAG_EXCHANGE) && P.tile > 4) {
        // balanced tiles of 4-site units, as many clusters as a tile of at
        // most E - 2*halo sites needs (so halo + keep + halo fits a cluster)
        const int64_t G = (d->n + (P.tile - 4) - 1) / (P.tile - 4);
        const int64_t units = d->n / 4;
        P.exchange = true;
        P.waves = G;
        P.uq = units / G;
        P.ur = units % G;
        P.tile = 4 * (P.uq + 1);          // the largest kept count
        P.zone = E - P.halo - 4 * P.uq;   // the left neighbour's right halo reaches this far
    }
    return P;
}

// Whether an exchange plan is well formed: at least 3 clusters and a chain
// longer than one cluster (so every halo site lies in a neighbour's kept
// sites, with one wrap at most), and every cluster keeps at least what its
// neighbours read (`halo` at its right end, `zone` at its left).
bool exchange_plan_ok(const Plan &P, int64_t n) {
    const int64_t E = 64 * static_cast<int64_t>(P.sites) * P.waves_per_cluster;
    return P.exchange && P.waves >= 3 && P.waves <= INT32_MAX && n > E && P.halo <= 4 * P.uq &&
           P.zone <= 4 * P.uq;
}

chain_rk4_plan public_plan(const chain_rk4_desc &d, const Plan &p) {
    chain_rk4_plan P{};
    P.method = d.method;
    P.resident = p.resident ? 1 : 0;
    P.sites_per_lane = p.sites;
    P.kdepth = p.depth;
    P.waves_per_cluster = p.waves_per_cluster;
    P.exchange = p.exchange ? 1 : 0;
    P.tile = p.tile;
    P.halo = p.halo;
    P.waves = p.waves;
    P.overlap_factor = p.tile > 0 ? 1.0 + 2.0 * double(p.halo) / double(p.tile) : 1.0;
    return P;
}


}  // namespace


namespace {

// Enqueue the passes of nsteps on stream s (`captured`: s is capturing a
// graph that will be replayed later).
int enqueue_steps(chain_rk4 *h, int64_t nsteps, hipStream_t s, bool captured) {
    const chain_rk4_desc &d = h->d;
    if (nsteps == 0) return CHAIN_OK;
    if (d.method == CHAIN_NAIVE && d.scheme == CHAIN_SCHEME_TABLEAU) {
        for (int64_t i = 0; i < nsteps; ++i) {
            hipError_t e = launch_naive_tableau_step(d.model, d.prec, h->front, h->naive_tab, d.n,
                                                     d.dt, h->tableau, s);
            if (e != hipSuccess) return hip_fail(e, "naive tableau step launch");
        }
        return CHAIN_OK;
    }
    if (d.method == CHAIN_NAIVE) {
        for (int64_t i = 0; i < nsteps; ++i) {
            hipError_t e = d.model == CHAIN_ROESSLER
                               ? launch_naive_roessler_step(h->front, h->naive, d.n, d.dt, s)
                               : launch_naive_step(d.model, d.prec, h->front, h->naive, d.n, d.dt, s);
            if (e != hipSuccess) return hip_fail(e, "naive step launch");
        }
        return CHAIN_OK;
    }
    if (h->plan.exchange && nsteps >= 2) {
        // one launch: an even number of passes of at most `depth` steps each
        int64_t passes = (nsteps + h->plan.depth - 1) / h->plan.depth;
        passes += passes % 2;
        if (passes > INT32_MAX) return fail(CHAIN_EINVAL, "too many steps in one call");
        const Plan &P = h->plan;
        // The progress counters keep counting over successive calls: every
        // cluster sets its counter after each pass but the last, so after a
        // call of `passes` passes all of them hold base + passes - 1, the next
        // call's base (also after a timed-out wait, which lets its cluster go
        // on). A call captured into a graph is replayed later, when the
        // counters have moved on: it clears them and starts from 0, and
        // every replay leaves the base unknown (step_graph), as does a base
        // near the top of the 32-bit range.
        int64_t base = h->xbase;
        if (captured || base < 0 || base + passes > (int64_t(1) << 30)) {
            hipError_t e =
                launch_fill_zero(h->xflags, static_cast<size_t>(P.waves) * sizeof(int32_t), s);
            if (e != hipSuccess) return hip_fail(e, "clearing the exchange flags");
            base = 0;
        }
        ExchangeRun a{h->front, h->back, d.n, P.uq, P.ur, P.halo, P.zone, nsteps, d.dt,
                      static_cast<int32_t>(P.waves), static_cast<int32_t>(passes), h->xflags,
                      h->xerror, kExchangeSpinLimit, static_cast<int32_t>(base)};
        hipError_t e = launch_exchange_roessler(P.sites, P.waves_per_cluster, a, s);
        if (e != hipSuccess) {
            h->xbase = -1;
            return hip_fail(e, "exchange launch");
        }
        h->xbase = captured ? -1 : base + passes - 1;
        return CHAIN_OK;
    }
    if (h->plan.resident) {
        ResidentRun r{h->front, h->front, d.n, d.dt, nsteps};
        hipError_t e = launch_resident(d.model, d.prec, r, s);
        if (e != hipSuccess) return hip_fail(e, "resident launch");
        return CHAIN_OK;
    }
    // Passes of `depth` steps; the pass count is made even (by splitting one
    // pass in two) so the state ends in the caller's buffers. Only when every
    // pass is a single step does an odd count remain; then the state is copied
    // back after the last pass.
    const int K = h->plan.depth;
    std::vector<int> ks(static_cast<size_t>(nsteps / K), K);
    if (nsteps % K) ks.push_back(static_cast<int>(nsteps % K));
    if (ks.size() % 2 == 1) {
        for (size_t i = ks.size(); i-- > 0;) {
            if (ks[i] >= 2) {
                const int a = ks[i] / 2, b = ks[i] - a;
                ks[i] = a;
                ks.insert(ks.begin() + static_cast<long>(i) + 1, b);
                break;
            }
        }
    }
    StateRef cur = h->front, nxt = h->back;
    for (int k : ks) {
        FusedPass a{cur, nxt, d.n, h->plan.tile, h->plan.halo, h->plan.waves, d.dt, k};
        hipError_t e =
            d.model == CHAIN_ROESSLER
                ? launch_fused_roessler(h->plan.sites, h->plan.waves_per_cluster, a, s)
            : d.scheme == CHAIN_SCHEME_TABLEAU
                ? launch_tableau(d.model, d.prec, h->plan.sites, h->plan.waves_per_cluster, a,
                                 h->tableau, s)
                : launch_fused(d.model, d.prec, h->plan.sites, h->plan.waves_per_cluster, a, s);
        if (e != hipSuccess) return hip_fail(e, "fused launch");
        std::swap(cur, nxt);
    }
    if (ks.size() % 2 == 1) {
        const size_t b = static_cast<size_t>(d.n) * elem_bytes(d.prec);
        HIP_TRY(hipMemcpyAsync(h->front.q, cur.q, b, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(h->front.p, cur.p, b, hipMemcpyDeviceToDevice, s));
        if (d.model == CHAIN_ROESSLER)
            HIP_TRY(hipMemcpyAsync(h->front.z, cur.z, b, hipMemcpyDeviceToDevice, s));
        if (has_carries(d.prec)) {
            const size_t cb = static_cast<size_t>(d.n) * carry_bytes(d.prec);
            HIP_TRY(hipMemcpyAsync(h->front.cq, cur.cq, cb, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(h->front.cp, cur.cp, cb, hipMemcpyDeviceToDevice, s));
        }
    }
    return CHAIN_OK;
}

int step_graph(chain_rk4 *h, int64_t nsteps) {
    auto it = h->graphs.find(nsteps);
    if (it == h->graphs.end()) {
        if (h->graphs.size() >= 8) {
            for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
            h->graphs.clear();
        }
        if (!h->capture) HIP_TRY(hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_steps(h, nsteps, h->capture, true);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(h->capture, &g);
        if (rc != CHAIN_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        it = h->graphs.emplace(nsteps, exec).first;
    }
    // a replayed exchange call leaves its counters at a value this handle
    // does not track: the next eager call clears them
    h->xbase = -1;
    HIP_TRY(hipGraphLaunch(it->second, h->stream));
    return CHAIN_OK;
}

}  // namespace

extern "C" {

size_t chain_rk4_workspace_bytes(const chain_rk4_desc *d) {
    if (check_desc(d) != CHAIN_OK) return 0;
    return layout(d).total;
}

int chain_rk4_create3(const chain_rk4_desc *d, void *q, void *p, void *z, void *workspace,
                      size_t ws_bytes, void *stream, chain_rk4 **out) {
    int rc = check_desc(d);
    if (rc != CHAIN_OK) return rc;
    if (!out) return fail(CHAIN_EINVAL, "out is NULL");
    *out = nullptr;
    const bool three = d->model == CHAIN_ROESSLER;
    if (!q || !p) return fail(CHAIN_EINVAL, "the coordinate arrays must be device pointers");
    if (three && !z) return fail(CHAIN_EINVAL, "the Roessler chain needs a z array");
    if (!three && z) return fail(CHAIN_EINVAL, "z must be NULL for a two-coordinate model");
    if ((reinterpret_cast<uintptr_t>(q) | reinterpret_cast<uintptr_t>(p) |
         reinterpret_cast<uintptr_t>(z)) & 15)
        return fail(CHAIN_EINVAL, "coordinate arrays must be 16-byte aligned");
    const Layout L = layout(d);
    if (ws_bytes < L.total)
        return fail(CHAIN_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    if (!workspace) return fail(CHAIN_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1))
        return fail(CHAIN_EINVAL, "workspace must be 256-byte aligned");

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (!is_gfx950(dev)) return fail(CHAIN_EDEVICE, "device %d is not a gfx950 GPU", dev);

    chain_rk4 *h = new (std::nothrow) chain_rk4();
    if (!h) return fail(CHAIN_ENOMEM, "out of host memory");
    char *ws = static_cast<char *>(workspace);
    h->d = *d;
    h->stream = static_cast<hipStream_t>(stream);
    h->plan = make_plan(d);
    h->front = StateRef{q, p, nullptr, nullptr, static_cast<double *>(z)};
    h->back = StateRef{nullptr, nullptr, nullptr, nullptr, nullptr};
    if (d->method == CHAIN_FUSED) {
        h->back.q = ws + L.back_q;
        h->back.p = ws + L.back_p;
        if (three) h->back.z = reinterpret_cast<double *>(ws + L.back_z);
    }
    if (has_carries(d->prec)) {
        h->front.cq = ws + L.cq;
        h->front.cp = ws + L.cp;
        if (d->method == CHAIN_FUSED) {
            h->back.cq = ws + L.back_cq;
            h->back.cp = ws + L.back_cp;
        }
    }
    if (d->method == CHAIN_NAIVE && d->scheme == CHAIN_SCHEME_TABLEAU) {
        NaiveTabBufs &b = h->naive_tab;
        int k = 0;
        for (int m = 0; m < kMaxStages - 1; ++m) b.kp[m] = ws + L.naive_tab[k++];
        b.qa = ws + L.naive_tab[k++];
        b.qb = ws + L.naive_tab[k++];
    } else if (d->method == CHAIN_NAIVE && !three) {
        // the per-stage kernels of the Hamiltonian chains: Q2/Q4, Q3, F1, F2
        // and the running force sum
        void **slots[kNaiveArraysHamiltonian] = {&h->naive.yaq, &h->naive.ybq, &h->naive.k1p,
                                                 &h->naive.k2p, &h->naive.k2q};
        for (int i = 0; i < kNaiveArraysHamiltonian; ++i) *slots[i] = ws + L.naive[i];
    } else if (d->method == CHAIN_NAIVE) {
        void **slots[10] = {&h->naive.k1q, &h->naive.k1p, &h->naive.k2q, &h->naive.k2p,
                            &h->naive.k3q, &h->naive.k3p, &h->naive.yaq, &h->naive.yap,
                            &h->naive.ybq, &h->naive.ybp};
        for (int i = 0; i < 10; ++i) *slots[i] = ws + L.naive[i];
        double **zs[5] = {&h->naive.k1z, &h->naive.k2z, &h->naive.k3z, &h->naive.yaz,
                          &h->naive.ybz};
        for (int i = 0; i < 5; ++i) *zs[i] = reinterpret_cast<double *>(ws + L.naive_z[i]);
    }
    h->partials = reinterpret_cast<double *>(ws + L.partials);
    h->result = reinterpret_cast<double *>(ws + L.result);
    if (d->flags & CHAIN_FLAG_EXCHANGE) {
        // every cluster must be held at once, one workgroup each
        const int cap = exchange_capacity_roessler(h->plan.sites, h->plan.waves_per_cluster);
        if (!exchange_plan_ok(h->plan, d->n) || cap < h->plan.waves) {
            const long long G = h->plan.waves;
            delete h;
            return fail(CHAIN_EINVAL,
                        "CHAIN_FLAG_EXCHANGE: %lld clusters for n = %lld; the device holds %d at "
                        "once, and the plan needs at least 3, each keeping the sites its "
                        "neighbours read",
                        G, (long long)d->n, cap);
        }
        h->xflags = reinterpret_cast<int32_t *>(ws + L.xflags);
        h->xerror = reinterpret_cast<int32_t *>(ws + L.xerror);
        hipError_t e = launch_fill_zero(h->xerror, sizeof(int32_t), h->stream);
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "clearing the exchange timeout word");
        }
    }
    if (has_carries(d->prec)) {
        const size_t cb = round_up(static_cast<size_t>(d->n) * carry_bytes(d->prec));
        hipError_t e = launch_fill_zero(h->front.cq, cb, h->stream);
        if (e == hipSuccess) e = launch_fill_zero(h->front.cp, cb, h->stream);
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "zeroing the carries");
        }
    }
    *out = h;
    return CHAIN_OK;
}

int chain_rk4_create(const chain_rk4_desc *d, void *q, void *p, void *workspace, size_t ws_bytes,
                     void *stream, chain_rk4 **out) {
    if (d && d->model == CHAIN_ROESSLER) {
        if (out) *out = nullptr;
        return fail(CHAIN_EINVAL, "the Roessler chain has three coordinates: use chain_rk4_create3");
    }
    return chain_rk4_create3(d, q, p, nullptr, workspace, ws_bytes, stream, out);
}

int chain_rk4_step(chain_rk4 *h, int64_t nsteps) {
    if (!h) return fail(CHAIN_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(CHAIN_EINVAL, "nsteps must be >= 0");
    if (h->d.scheme == CHAIN_SCHEME_TABLEAU && !h->has_tableau)
        return fail(CHAIN_EINVAL, "no tableau set (chain_rk4_set_tableau)");
    if (nsteps == 0) return CHAIN_OK;
    if (h->d.flags & CHAIN_FLAG_GRAPH) return step_graph(h, nsteps);
    return enqueue_steps(h, nsteps, h->stream, false);
}

int chain_rk4_energy(chain_rk4 *h, double *e_out) {
    if (!h || !e_out) return fail(CHAIN_EINVAL, "handle and e_out must be non-NULL");
    if (h->d.model == CHAIN_ROESSLER)
        return fail(CHAIN_EINVAL, "the Roessler chain has no conserved energy");
    hipError_t e = launch_energy(h->d.model, h->d.prec, h->front, h->d.n, h->partials, h->result,
                                 h->stream);
    if (e != hipSuccess) return hip_fail(e, "energy launch");
    double v = 0.0;
    HIP_TRY(hipMemcpyAsync(&v, h->result, sizeof v, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    *e_out = v;
    if (!std::isfinite(v)) return fail(CHAIN_ENONFINITE, "energy is not finite (%g)", v);
    return CHAIN_OK;
}

int chain_rk4_set_stream(chain_rk4 *h, void *stream) {
    if (!h) return fail(CHAIN_EINVAL, "handle is NULL");
    h->stream = static_cast<hipStream_t>(stream);
    return CHAIN_OK;
}

int chain_rk4_get_plan(const chain_rk4 *h, chain_rk4_plan *out) {
    if (!h || !out) return fail(CHAIN_EINVAL, "handle and out must be non-NULL");
    *out = public_plan(h->d, h->plan);
    return CHAIN_OK;
}

int chain_rk4_get_carries(const chain_rk4 *h, void **cq, void **cp) {
    if (!h || !cq || !cp) return fail(CHAIN_EINVAL, "handle, cq and cp must be non-NULL");
    *cq = h->front.cq;
    *cp = h->front.cp;
    return CHAIN_OK;
}

namespace {

int check_tableau(const chain_rk4_tableau *t, TabArgs *out) {
    if (!t) return fail(CHAIN_EINVAL, "tableau is NULL");
    if (t->stages < 1 || t->stages > CHAIN_MAX_STAGES)
        return fail(CHAIN_EINVAL, "stages must be 1..%d (got %d)", CHAIN_MAX_STAGES, t->stages);
    if (t->reserved != 0) return fail(CHAIN_EINVAL, "tableau reserved must be 0");
    static_assert(CHAIN_MAX_STAGES == kMaxStages, "stage bound");
    TabArgs a{};
    a.stages = t->stages;
    for (int j = 0; j < t->stages; ++j) {
        for (int m = 0; m < j; ++m) {
            if (!std::isfinite(t->a[j][m])) return fail(CHAIN_EINVAL, "a[%d][%d] is not finite", j, m);
            a.a[j][m] = t->a[j][m];
        }
        if (!std::isfinite(t->b[j])) return fail(CHAIN_EINVAL, "b[%d] is not finite", j);
        a.b[j] = t->b[j];
    }
    *out = a;
    return CHAIN_OK;
}

// The coefficients the kernels use (TabArgs), for step h, in FP64 and in a
// fixed order: with P_m = p + h sum_l a_ml F_l the stage arguments are
// Q_j = q + h sum_m a_jm P_m = q + h c_j p + h^2 sum_l (A^2)_jl F_l, and the
// update q' = q + h sum_m b_m P_m = q + h (sum b) p + h^2 sum_l (b^T A)_l F_l.
void derive_tableau(TabArgs &t, double h) {
    const int s = t.stages;
    t.hsb = 0.0;
    for (int j = 0; j < kMaxStages; ++j) {
        double c = 0.0, w = 0.0;
        for (int m = 0; m < j; ++m) c += t.a[j][m];
        for (int m = j + 1; m < s; ++m) w += t.b[m] * t.a[m][j];
        t.hc[j] = j < s ? h * c : 0.0;
        t.hb[j] = j < s ? h * t.b[j] : 0.0;
        t.w[j] = j < s ? h * h * w : 0.0;
        if (j < s) t.hsb += t.b[j];
        for (int l = 0; l < kMaxStages; ++l) {
            double g = 0.0;
            for (int m = l + 1; m < j; ++m) g += t.a[j][m] * t.a[m][l];
            t.g[j][l] = (j < s && l < s) ? h * h * g : 0.0;
        }
    }
    t.hsb *= h;
}

// Plan of a tableau method: the halo covers the tableau's exact reach.
int tableau_plan(const chain_rk4_desc *d, const TabArgs &a, Plan *out) {
    const int64_t reach = std::max<int64_t>(1, tableau_reach_of(a, model_range(d->model)));
    Plan P = make_plan(d, reach, a.stages);
    if (d->method == CHAIN_FUSED && !tableau_shape_ok(a.stages, P.sites, P.waves_per_cluster))
        return fail(CHAIN_EINVAL,
                    "the tableau kernel runs sites_per_lane 4 or 8 (4 beyond 4 stages) and "
                    "waves_per_cluster 1 or 4 (got %d, %d for %d stages)",
                    P.sites, P.waves_per_cluster, a.stages);
    if (d->method == CHAIN_FUSED && P.tile < 1)
        return fail(CHAIN_EINVAL, "the cluster is too small for this tableau's reach");
    *out = P;
    return CHAIN_OK;
}

}  // namespace

int64_t chain_rk4_tableau_reach(int32_t model, const chain_rk4_tableau *t) {
    TabArgs a;
    if (model != CHAIN_QUARTIC && model != CHAIN_HARMONIC && model != CHAIN_QUARTIC_NNN &&
        model != CHAIN_HARMONIC_NNN)
        return -1;
    if (check_tableau(t, &a) != CHAIN_OK) return -1;
    return tableau_reach_of(a, model_range(model));
}

int chain_rk4_set_tableau(chain_rk4 *h, const chain_rk4_tableau *t) {
    if (!h) return fail(CHAIN_EINVAL, "handle is NULL");
    if (h->d.scheme != CHAIN_SCHEME_TABLEAU)
        return fail(CHAIN_EINVAL, "the handle was not created with CHAIN_SCHEME_TABLEAU");
    TabArgs a;
    int rc = check_tableau(t, &a);
    if (rc != CHAIN_OK) return rc;
    Plan P;
    rc = tableau_plan(&h->d, a, &P);
    if (rc != CHAIN_OK) return rc;
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    derive_tableau(a, h->d.dt);
    h->tableau = a;
    h->plan = P;
    h->has_tableau = true;
    return CHAIN_OK;
}

int chain_rk4_plan_for(const chain_rk4_desc *d, const chain_rk4_tableau *t,
                       chain_rk4_plan *out) {
    if (!out) return fail(CHAIN_EINVAL, "out is NULL");
    int rc = check_desc(d);
    if (rc != CHAIN_OK) return rc;
    Plan P;
    if (d->scheme == CHAIN_SCHEME_TABLEAU) {
        if (!t) return fail(CHAIN_EINVAL, "a CHAIN_SCHEME_TABLEAU descriptor needs its tableau");
        TabArgs a;
        rc = check_tableau(t, &a);
        if (rc == CHAIN_OK) rc = tableau_plan(d, a, &P);
        if (rc != CHAIN_OK) return rc;
    } else {
        if (t) return fail(CHAIN_EINVAL, "a tableau is only given with CHAIN_SCHEME_TABLEAU");
        P = make_plan(d);
        if ((d->flags & CHAIN_FLAG_EXCHANGE) && !exchange_plan_ok(P, d->n))
            return fail(CHAIN_EINVAL, "CHAIN_FLAG_EXCHANGE: the chain needs at least 3 clusters, "
                                      "each keeping the sites its neighbours read");
    }
    *out = public_plan(*d, P);
    return CHAIN_OK;
}

int chain_rk4_check(chain_rk4 *h) {
    if (!h) return fail(CHAIN_EINVAL, "handle is NULL");
    if (!h->xerror) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        return CHAIN_OK;
    }
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, h->xerror, sizeof err, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (err == 0) return CHAIN_OK;
    hipError_t e = launch_fill_zero(h->xerror, sizeof(int32_t), h->stream);
    if (e != hipSuccess) return hip_fail(e, "clearing the exchange timeout word");
    HIP_TRY(hipStreamSynchronize(h->stream));
    return fail(CHAIN_ETIMEOUT, "a cluster's wait for its neighbours timed out");
}

int chain_rk4_destroy(chain_rk4 *h) {
    if (!h) return CHAIN_OK;
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    if (h->capture) (void)hipStreamDestroy(h->capture);
    delete h;
    return CHAIN_OK;
}

const char *chain_rk4_strerror(int status) {
    switch (status) {
    case CHAIN_OK: return "success";
    case CHAIN_EINVAL: return "invalid argument";
    case CHAIN_ENOMEM: return "workspace too small";
    case CHAIN_EHIP: return "HIP runtime error";
    case CHAIN_ENONFINITE: return "energy is not finite";
    case CHAIN_EDEVICE: return "device is not a gfx950 GPU";
    case CHAIN_ETIMEOUT: return "a batched launch timed out waiting for a neighbour";
    default: return "unknown status";
    }
}

const char *chain_rk4_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
