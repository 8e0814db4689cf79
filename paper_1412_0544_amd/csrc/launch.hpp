// launch.hpp -- internal interface between the host library and the kernel
// translation units. Each kernel file exposes plain host launchers; nothing
// here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chainrk4 {

// Buffers of one chain's state. FP64: q, p are double*. FP32 with compensated
// update: q, p are float* and cq, cp are the float carries.
struct StateRef {
    void *q, *p;
    void *cq, *cp;   // compensated update: per-site carries (float, or double for
                     // FP32 state with FP64 carries)
    double *z;   // third coordinate of the Roessler chain (q = x, p = y)
};

// One pass of the fused kernel: every cluster (W wavefronts) owns `tile`
// output sites and recomputes `halo` sites on each side, advancing
// `ksteps` <= halo / reach steps (reach: sites a step's edge error travels,
// 2 for the NN chains, 4 for the NNN and Roessler chains). `waves` counts
// clusters.
struct FusedPass {
    StateRef in, out;
    int64_t n;
    int64_t tile;
    int64_t halo;
    int64_t waves;
    double dt;
    int ksteps;
    int balance;  // set by the launcher: every cluster resident at once, so
                  // wavefronts take issue priority by progress
};

// Whole-ring resident run: one workgroup holds the chain on chip for nsteps.
struct ResidentRun {
    StateRef in, out;  // out may equal in
    int64_t n;
    double dt;
    int64_t nsteps;
};

// Naive method: one kernel per RK stage over memory. The Roessler chain uses
// every array (slopes k1..k3 and the ping-pong stage arguments of x, y, z);
// the Hamiltonian chains use yaq (Q2, then Q4), ybq (Q3), k1p (F1), k2p (F2)
// and k2q (the running sum of the forces).
struct NaiveBufs {
    void *k1q, *k1p, *k2q, *k2p, *k3q, *k3p;  // stage slopes
    void *yaq, *yap, *ybq, *ybp;              // stage arguments (ping-pong)
    double *k1z, *k2z, *k3z, *yaz, *ybz;      // Roessler: third coordinate
};

// Resident rings: one workgroup of 256 threads up to 256 sites, else 1024
// threads (16 wavefronts hide the LDS and barrier latency of each stage far
// better than 4: 2.3x faster per step at 1024 sites), up to 4 sites each.
constexpr int kResidentThreadsSmall = 256;
constexpr int kResidentThreads = 1024;
constexpr int kResidentMaxSites = 4096;
constexpr int kFusedThreads = 256;        // 4 one-wavefront clusters per block

hipError_t launch_fused(int model, int prec, int sites_per_lane, int waves_per_cluster,
                        const FusedPass &a, hipStream_t s);
hipError_t launch_resident(int model, int prec, const ResidentRun &a, hipStream_t s);
hipError_t launch_naive_step(int model, int prec, StateRef y, const NaiveBufs &b, int64_t n,
                             double dt, hipStream_t s);

// Explicit Runge-Kutta by Butcher tableau: coefficients a[j][m] (m < j) and
// weights b[m] of `stages` <= kMaxStages stages.
constexpr int kMaxStages = 8;
struct TabArgs {
    int32_t stages, pad;
    double a[kMaxStages][kMaxStages];
    double b[kMaxStages];
    // What the kernels use, derived in FP64 for the handle's step h (for
    // dq/dt = p the q stage arguments and the q update follow from p and the
    // forces): Q_j = q + hc_j p + sum_l g_jl F_l, p' = p + sum_m hb_m F_m,
    // q' = q + hsb p + sum_l w_l F_l.
    double hc[kMaxStages];             // h c_j, c_j = sum_m a_jm
    double g[kMaxStages][kMaxStages];  // h^2 (A^2)_jl (zero for l >= j - 1)
    double hb[kMaxStages];             // h b_m
    double w[kMaxStages];              // h^2 (b^T A)_l (zero for the last stage)
    double hsb;                        // h sum_m b_m
};
// Cluster shapes the tableau kernel is built for: sites per lane 4 or 8 with
// up to 4 stages, 4 with up to 8; wavefronts per cluster 1 or 4.
hipError_t launch_tableau(int model, int prec, int sites_per_lane, int waves_per_cluster,
                          const FusedPass &a, const TabArgs &t, hipStream_t s);

// The per-stage implementation of a tableau method (Sec. 2.2 with general
// coefficients): kernel j evaluates the force F_j at its stage argument and
// forms the next argument (or, for the last stage, the new state in place).
// The forces of stages m < s-1 go through memory.
struct NaiveTabBufs {
    void *kp[kMaxStages - 1];  // F(Q_m), m = 0..s-2
    void *qa, *qb;             // stage arguments (ping-pong)
};
hipError_t launch_naive_tableau_step(int model, int prec, StateRef y, const NaiveTabBufs &b,
                                     int64_t n, double dt, const TabArgs &t, hipStream_t s);

// Roessler chain (FP64): fused cluster pass and the per-stage baseline.
constexpr int kModelRoessler = 2;
hipError_t launch_fused_roessler(int sites_per_lane, int waves_per_cluster, const FusedPass &a,
                                 hipStream_t s);

// A whole step call with every cluster held in registers: one workgroup per
// cluster for all passes of the call. Between passes a cluster writes the
// kept sites its two neighbours read into that pass's exchange buffer
// (device-coherent stores), marks the pass done, waits for its neighbours
// and reloads its halo from their kept sites. Every cluster must be resident
// at once. Clusters keep balanced tiles of 4-site units, as in a batch.
struct ExchangeRun {
    StateRef front, back;   // front: the caller's buffers (initial and final
                            // state); pass j exchanges through front (j odd)
                            // or back (j even)
    int64_t n;
    int64_t uq, ur;         // cluster g keeps 4*uq sites, 4*(uq+1) if g < ur;
                            // the last one also the n % 4 remainder
    int64_t halo;           // recomputed sites per side, >= reach * steps of a pass
    int64_t zone;           // kept sites at a cluster's left end that its left
                            // neighbour reads (its right halo reaches that far)
    int64_t steps;          // steps of the call: pass j advances steps / passes,
                            // one more if j < steps % passes
    double dt;
    int32_t clusters;       // >= 3
    int32_t passes;         // even, >= 2 (the last pass ends in front)
    int32_t *flags;         // per cluster: base + passes done
    int32_t *error;         // set if a bounded wait expires (never cleared here)
    int32_t spin_limit;     // polls before a wait gives up
    int32_t base;           // every flag's value when the launch starts
};
hipError_t launch_exchange_roessler(int sites_per_lane, int waves_per_cluster,
                                    const ExchangeRun &a, hipStream_t s);
// Clusters of that shape the current device holds at once (0 on error).
int exchange_capacity_roessler(int sites_per_lane, int waves_per_cluster);
hipError_t launch_naive_roessler_step(StateRef y, const NaiveBufs &b, int64_t n, double dt,
                                      hipStream_t s);

// Energy: per-block FP64 partials, then one fixed-order finishing block.
constexpr int kEnergyThreads = 256;
constexpr int kEnergyMaxBlocks = 1024;
int energy_blocks(int64_t n);
hipError_t launch_energy(int model, int prec, StateRef y, int64_t n, double *partials,
                         double *result, hipStream_t s);

hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t s);

// ---------------------------------------------------------------------------
// Batches: one persistent launch over many chains. Work items, claimed in
// increasing order from a counter: first one item per resident chain (a ring
// short enough to stay in LDS for all its steps), then, pass by pass, the
// cluster items. A chain is cut into wide clusters (all kBatchWaves
// wavefronts of a workgroup, 64*S*kBatchWaves sites) followed by at most
// three narrow ones (one wavefront, 64*S sites), whichever mix holds it in
// the fewest lane-sites. An item is one wide cluster, or a pack of up to
// kBatchWaves narrow clusters (of consecutive chains), one per wavefront.
// Cluster g of chain c at pass e needs clusters g-1, g, g+1 of chain c to
// have finished pass e-1; those items have smaller indices, so waiting on
// them cannot deadlock.
// ---------------------------------------------------------------------------
constexpr int kBatchThreads = 256;      // 4 wavefronts: one wide cluster
constexpr int kBatchWaves = 4;
constexpr int kBatchResidentSites = 1024;  // longest ring a batch keeps on chip
constexpr int kMaxNarrow = 3;              // narrow clusters per chain at most
// item_chain[kBatchWaves * w + 1] of a wide item (slot 0 holds its cluster);
// an empty slot of a narrow pack holds kEmptySlot
constexpr int32_t kWideItem = -2;
constexpr int32_t kEmptySlot = -1;

constexpr int batch_resident_max(int /*prec*/) { return kBatchResidentSites; }

struct BatchChain {
    StateRef front, back;
    int64_t n;
    int64_t nsteps;        // resident chains: steps of this launch
    int64_t uq, ur;        // tiled: wide cluster i keeps 4*(uq + (i < ur)) sites
    double dt;
    int32_t clusters;      // tiled: clusters per pass, wide ones first
    int32_t passes;        // tiled: passes of this launch
    int32_t head0, head1;  // steps of passes 0 and 1 when nhead == 2
    int32_t nhead;         // 0 or 2
    int32_t tail;          // steps of the last pass, 0 if it is a full pass
    int32_t flag_base;     // first progress flag of this chain
    int32_t wide;          // tiled: wide clusters; the rest are narrow
    int32_t nuq, nur;      // narrow cluster j keeps 4*(nuq + (j < nur)) sites;
                           // the chain's last cluster also the n % 4 remainder
};

struct BatchArgs {
    const BatchChain *chains;      // tiled chains (by passes, descending), then resident
    const int64_t *pass_off;       // pass_off[e]: first tiled item of pass e
    const int32_t *item_chain;     // kBatchWaves slots per item: chain of each
    const int32_t *item_cluster;   // cluster of each slot
    int32_t *flags;                // per cluster: passes completed
    unsigned long long *counter;   // next unclaimed item
    int32_t *error;                // set when a bounded wait expires
    int64_t total_items;
    int64_t halo;                  // 2 * depth, rounded up to 4
    int32_t n_resident, n_tiled;
    int32_t max_passes;
    int32_t depth;                 // steps of a full pass
    int32_t spin_limit;            // polls before a wait gives up
    int32_t fences;                // hand-off by cache write-back/invalidate
};

// Blocks of the persistent kernel the device holds at once (0 on error).
int persistent_capacity(int model, int prec, int sites_per_lane, bool resident_items);
hipError_t launch_persistent(int model, int prec, int sites_per_lane, int blocks,
                             const BatchArgs &a, hipStream_t s);

}  // namespace chainrk4
