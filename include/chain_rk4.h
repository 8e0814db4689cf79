/*
 * chain_rk4.h -- C ABI of the MI355X (gfx950) library that advances large
 * periodic one-dimensional chains with classical explicit RK4.
 *
 * The problem (Mulansky, "Optimizing Large-Scale ODE Simulations"):
 *   a ring of N sites with state r_i = (q_i, p_i), a homogeneous
 *   nearest-neighbour vector field (Sec. 2.1 Eq. 2), periodic boundary
 *   (Sec. 3.1), advanced by RK4 with a fixed step dt (Sec. 2.2 Eq. 3-5):
 *     dq_i/dt = p_i,   dp_i/dt = F_i(q_{i-1}, q_i, q_{i+1})
 *   quartic:  F_i = -(q_i + q_i^3) + (q_{i+1} - q_i)^3 - (q_i - q_{i-1})^3
 *   harmonic: F_i = -q_i + (q_{i+1} - 2 q_i + q_{i-1})
 * the same two with next-nearest-neighbour bonds (the generalisation named in
 * Sec. 5; every site also bonded to its second neighbours, same potential):
 *   quartic NNN:  F_i += (q_{i+2} - q_i)^3 - (q_i - q_{i-2})^3
 *   harmonic NNN: F_i += (q_{i+2} - 2 q_i + q_{i-2})
 * and the paper's own test system, the Roessler chain (Sec. 3.1 Eq. 6-7),
 * three coordinates per site with a = 0.2, b = 1, c = 9:
 *   dx_i/dt = -y_i - z_i + (x_{i+1} - 2 x_i + x_{i-1})
 *   dy_i/dt = x_i + a y_i,   dz_i/dt = b + z_i (x_i - c)
 *
 * Conventions for every call:
 *   - Device pointers are HIP device memory of the current device; host
 *     pointers are ordinary host memory. The library never frees memory it
 *     did not allocate.
 *   - A stream argument is a hipStream_t passed as void*; NULL is the null
 *     stream. Work is enqueued on that stream and calls return before it runs
 *     unless stated otherwise.
 *   - Every call returns a chain_status. Arguments are validated before any
 *     HIP call, so an invalid argument has no side effect. A HIP failure
 *     returns CHAIN_EHIP; chain_rk4_last_error() then gives the message.
 *   - Handles are not thread-safe; distinct handles are independent.
 *   - Results are bit-identical for every tile size, temporal depth, method
 *     and batch placement of the FP64 path, and likewise of the FP32 path.
 */
#ifndef CHAIN_RK4_H
#define CHAIN_RK4_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chain_rk4 chain_rk4;
typedef struct chain_rk4_batch chain_rk4_batch;

enum chain_model {
    CHAIN_QUARTIC = 0,   /* quartic on-site and bond potentials (formula above) */
    CHAIN_HARMONIC = 1,  /* the linear chain (formula above) */
    CHAIN_ROESSLER = 2,  /* the Roessler chain (formula above): FP64 only,
                            created with chain_rk4_create3, no energy, no
                            batches, never kept resident on chip */
    CHAIN_QUARTIC_NNN = 3, /* quartic chain with second-neighbour bonds; no
                              batches, never kept resident on chip */
    CHAIN_HARMONIC_NNN = 4 /* harmonic chain with second-neighbour bonds; the
                              same restrictions */
};

enum chain_prec {
    CHAIN_FP64 = 0,        /* q, p and every stage in FP64 */
    CHAIN_FP32_KAHAN = 1,  /* q, p and stages in FP32; the final update of each
                              step is Kahan-compensated with a per-site FP32
                              carry; energies are reduced in FP64 */
    CHAIN_FP32_KAHAN64 = 2,/* as CHAIN_FP32_KAHAN with FP64 carries: the
                              increment (h/6)*sum and the carry are FP64, q and
                              p stay FP32. Quartic and harmonic chains (NN and
                              NNN), classical RK4 on single handles; no
                              resident rings, tableaus or batches */
    CHAIN_FP32 = 3         /* plain FP32, no compensation: the control against
                              which the compensated forms are measured; the
                              same restrictions as CHAIN_FP32_KAHAN64 */
};

enum chain_method {
    CHAIN_FUSED = 0,  /* one pass over memory per `kdepth` steps: each tile is
                         extended by reach*kdepth sites per side that are
                         recomputed and discarded (Sec. 2.3, the overlap per
                         side per step, carried over several steps). reach is
                         2 for the quartic and harmonic chains (dq/dt = p is
                         local, so an edge error advances one site per two
                         stages), 4 for the NNN and Roessler chains */
    CHAIN_NAIVE = 1   /* the standard implementation: one kernel per RK stage,
                         every stage result goes through memory (Sec. 2.2) */
};

enum chain_scheme {
    CHAIN_SCHEME_RK4 = 0,     /* classical RK4 (Sec. 2.2: c = (0, 1/2, 1/2, 1),
                                 a21 = a32 = 1/2, a43 = 1, b = (1/6, 1/3, 1/3,
                                 1/6)) on the dedicated kernels */
    CHAIN_SCHEME_TABLEAU = 1  /* any explicit Runge-Kutta method, given by
                                 chain_rk4_set_tableau before the first step
                                 (Sec. 2.2 Eq. 3-5 with general coefficients;
                                 the paper notes the technique applies to every
                                 explicit scheme). The quartic, harmonic
                                 and NNN models; CHAIN_NAIVE runs one
                                 kernel per stage with every slope in the
                                 workspace (18 arrays of n values) */
};

#define CHAIN_MAX_STAGES 8

/* Butcher tableau of an explicit method with `stages` stages. Stage j
 * (0-based) evaluates the field at r + dt * sum_{m<j} a[j][m] k_m; the step
 * ends with r + dt * sum_{m<stages} b[m] k_m. Entries a[j][m] with m >= j or
 * j >= stages, and b[m] with m >= stages, are ignored. The models are
 * autonomous, so no nodes c are needed. */
typedef struct chain_rk4_tableau {
    int32_t stages;          /* 1..CHAIN_MAX_STAGES */
    int32_t reserved;        /* must be 0 */
    double a[CHAIN_MAX_STAGES][CHAIN_MAX_STAGES];
    double b[CHAIN_MAX_STAGES];
} chain_rk4_tableau;

enum chain_flags {
    CHAIN_FLAG_GRAPH = 1,        /* replay each distinct step count from a
                                    captured hipGraph instead of launching pass
                                    by pass */
    CHAIN_FLAG_NO_RESIDENT = 2,  /* always run the tiled passes (the default
                                    since the tiled plan measured faster at
                                    every length; kept for compatibility) */
    CHAIN_FLAG_RESIDENT = 4,     /* keep a quartic or harmonic ring of at most
                                    4096 sites resident on chip in one
                                    workgroup for all steps of a call (one
                                    launch per call, stage arguments in
                                    LDS); CHAIN_EINVAL for longer rings,
                                    other models or schemes, or together
                                    with CHAIN_FLAG_NO_RESIDENT */
    CHAIN_FLAG_EXCHANGE = 8      /* Roessler chain, fused method: a step call
                                    of two or more steps holds every cluster
                                    in registers for all its passes (one
                                    workgroup each, one launch per call);
                                    between passes a cluster writes only the
                                    kept sites its two neighbours read and
                                    reloads its halo from theirs, instead of
                                    storing and loading every site (the
                                    overlap of Sec. 2.3 renewed from memory,
                                    not the whole cluster). Same results bit
                                    for bit. The whole chain must be held at
                                    once: chain_rk4_create returns
                                    CHAIN_EINVAL if it needs more clusters
                                    than the device holds, fewer than 3, or
                                    is no longer than a cluster. Default
                                    kdepth 13 (edge swaps are cheaper than
                                    deeper overlap). Progress counters in the
                                    workspace carry over from call to call;
                                    a graph-captured call clears them first */
};

typedef enum chain_status {
    CHAIN_OK = 0,
    CHAIN_EINVAL = -1,      /* invalid argument (nothing was done) */
    CHAIN_ENOMEM = -2,      /* workspace too small */
    CHAIN_EHIP = -3,        /* a HIP runtime call failed */
    CHAIN_ENONFINITE = -4,  /* an energy came out NaN or infinite */
    CHAIN_EDEVICE = -5,     /* the current device is not a gfx950 GPU */
    CHAIN_ETIMEOUT = -6     /* a batched launch hit its bounded wait */
} chain_status;

typedef struct chain_rk4_desc {
    int64_t n;               /* sites on the ring, >= 1 (N = 1, 2 are legal) */
    int32_t model;           /* enum chain_model */
    int32_t prec;            /* enum chain_prec */
    double dt;               /* step size; finite, may be negative (reversal) */
    int32_t method;          /* enum chain_method */
    int32_t sites_per_lane;  /* fused: sites per GPU lane, 0 = default, else
                                2, 4, 8 or 16; 6 for classical RK4 of the
                                FP64 quartic and harmonic chains;
                                CHAIN_ROESSLER takes 4, 6, 8 or 16 (4, 6 or 8
                                with CHAIN_FLAG_EXCHANGE); the tableau kernel
                                takes 4 or 8 */
    int32_t kdepth;          /* fused: RK4 steps per pass over memory, 0 =
                                default, else 1..32 */
    int32_t waves_per_cluster; /* fused: wavefronts that share one cluster
                                (edge values through LDS), 0 = default,
                                else 1, 2, 4 or 8 */
    int32_t flags;           /* enum chain_flags, or 0 */
    int32_t scheme;          /* enum chain_scheme (0 = classical RK4) */
} chain_rk4_desc;

/* Plan chosen for a handle: what one step call launches. */
typedef struct chain_rk4_plan {
    int32_t method, sites_per_lane, kdepth, resident; /* resident: 1 if the
                                    whole ring stays on chip for all steps */
    int32_t waves_per_cluster;
    int32_t exchange;            /* 1 if step calls hold every cluster in
                                    registers and exchange edge sites
                                    (CHAIN_FLAG_EXCHANGE); tile is then the
                                    largest kept count of a cluster */
    int64_t tile;                /* output sites per cluster and pass */
    int64_t halo;                /* recomputed sites per side: reach * kdepth
                                    rounded up to a whole 16-byte vector of the
                                    state (2 FP64 or 4 FP32 sites), so every
                                    cluster starts on a 16-byte boundary */
    int64_t waves;               /* clusters per pass */
    double overlap_factor;       /* sites computed / sites kept per pass,
                                    1 + 2*halo/tile (Sec. 2.3) */
} chain_rk4_plan;

/*
 * Device workspace bytes a chain described by `d` needs (the back buffer of
 * the ping-pong update, the carries of the compensated FP32 precisions, the
 * naive method's stage arrays and the energy partials). Returns 0 if `d` is
 * invalid.
 */
size_t chain_rk4_workspace_bytes(const chain_rk4_desc *d);

/*
 * Create a handle over caller-owned device buffers.
 *   q, p       device arrays of d->n values (double for CHAIN_FP64, float for
 *              the FP32 precisions), 16-byte aligned; they hold the initial state
 *              and, after each step call completes, the advanced state.
 *   workspace  device buffer of ws_bytes >= chain_rk4_workspace_bytes(d),
 *              256-byte aligned (NULL allowed only if that size is 0).
 *   stream     stream for every later call on this handle.
 * The handle borrows q, p and workspace until chain_rk4_destroy. The carries
 * of a compensated FP32 precision are zeroed on `stream`. Returns CHAIN_EINVAL for NULL or misaligned
 * pointers or an invalid descriptor, CHAIN_ENOMEM if ws_bytes is too small,
 * CHAIN_EDEVICE if the current device is not gfx950.
 */
int chain_rk4_create(const chain_rk4_desc *d, void *q, void *p, void *workspace,
                     size_t ws_bytes, void *stream, chain_rk4 **out);

/*
 * Create a handle over three caller-owned coordinate arrays: x, y, z of the
 * Roessler chain (d->model == CHAIN_ROESSLER, d->prec == CHAIN_FP64), each
 * d->n doubles, 16-byte aligned; the other arguments as chain_rk4_create.
 * For the two-coordinate models z must be NULL and the call is the same as
 * chain_rk4_create(d, x, y, ...). chain_rk4_create rejects CHAIN_ROESSLER
 * with CHAIN_EINVAL.
 */
int chain_rk4_create3(const chain_rk4_desc *d, void *x, void *y, void *z, void *workspace,
                      size_t ws_bytes, void *stream, chain_rk4 **out);

/* Enqueue nsteps (>= 0) RK4 steps on the handle's stream (asynchronous). */
int chain_rk4_step(chain_rk4 *h, int64_t nsteps);

/*
 * Total energy of the current state, in FP64, written to *e_out (host).
 * Quartic: sum_i p_i^2/2 + q_i^2/2 + q_i^4/4 + (q_{i+1}-q_i)^4/4;
 * harmonic: sum_i p_i^2/2 + q_i^2/2 + (q_{i+1}-q_i)^2/2; the NNN models add
 * (q_{i+2}-q_i)^4/4 or (q_{i+2}-q_i)^2/2 per site. For the compensated FP32
 * precisions each coordinate enters as (hi - carry) in FP64. The sum order is fixed for
 * a given n, so repeated calls agree bitwise. Synchronises the stream.
 * Returns CHAIN_ENONFINITE (with *e_out set) if the energy is NaN or Inf,
 * CHAIN_EINVAL for a CHAIN_ROESSLER handle (a dissipative system with no
 * conserved energy).
 */
int chain_rk4_energy(chain_rk4 *h, double *e_out);

/*
 * For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc): the energy of chain_rk4_energy for a
 * state in caller buffers, with no handle and no workspace.
 *   model  CHAIN_QUARTIC, CHAIN_HARMONIC, CHAIN_QUARTIC_NNN or
 *          CHAIN_HARMONIC_NNN; prec any enum chain_prec.
 *   n      sites, 1..2^40 (CHAIN_EINVAL beyond).
 *   q, p   device arrays of n values (double for CHAIN_FP64, float else),
 *          16-byte aligned; read only.
 *   cq, cp the carries of a compensated FP32 state (n floats, or n doubles
 *          for CHAIN_FP32_KAHAN64; each coordinate enters as hi - carry),
 *          NULL for CHAIN_FP64 and CHAIN_FP32.
 *   stream where the kernels run; the call synchronises it.
 * The result is the same bits as chain_rk4_energy of a handle over the same
 * buffers. The partial sums live in a device array the library owns (1024
 * partials and the result, about 8.4 KB on each GPU it runs on, kept until the
 * process ends); the call allocates nothing. Calls that overlap on one GPU
 * share that array and race. Returns CHAIN_ENONFINITE (with *e_out set) for a
 * NaN or infinite energy, CHAIN_EDEVICE on a device other than gfx950.
 */
int chain_rk4_energy_noalloc(int32_t model, int32_t prec, int64_t n, const void *q,
                             const void *p, const void *cq, const void *cp, void *stream,
                             double *e_out);

/* Replace the stream used by later calls on this handle. */
int chain_rk4_set_stream(chain_rk4 *h, void *stream);

/* Report the plan of a handle (host struct). */
int chain_rk4_get_plan(const chain_rk4 *h, chain_rk4_plan *out);

/*
 * The plan chain_rk4_create (and, for CHAIN_SCHEME_TABLEAU, a following
 * chain_rk4_set_tableau with tableau `t`) would give descriptor `d`, without
 * a GPU or a handle: the granularity of Sec. 2.3 the library picks for this
 * chain. `t` must be given for CHAIN_SCHEME_TABLEAU and be NULL otherwise.
 * Returns CHAIN_EINVAL where create or set_tableau would.
 */
int chain_rk4_plan_for(const chain_rk4_desc *d, const chain_rk4_tableau *t,
                       chain_rk4_plan *out);

/*
 * Device pointers of the per-site carries (n floats each, or n doubles for
 * CHAIN_FP32_KAHAN64, inside the workspace) that complete the state of a
 * compensated FP32 handle: the compensated coordinate is q - cq, the momentum
 * p - cp. Copying q, p and both carries saves the full state; writing them
 * restores it. For CHAIN_FP64 and CHAIN_FP32 (no carries) both pointers are
 * set to NULL.
 */
int chain_rk4_get_carries(const chain_rk4 *h, void **cq, void **cp);

/*
 * Give a CHAIN_SCHEME_TABLEAU handle its method (copied; it may be set again
 * between step calls). Validation: 1 <= stages <= CHAIN_MAX_STAGES, finite
 * coefficients, and for CHAIN_FUSED a cluster shape the tableau kernel is
 * built for (sites_per_lane 4 or 8 for up to 4 stages, 4 beyond;
 * waves_per_cluster 1 or 4). The halo becomes reach * kdepth with reach from
 * chain_rk4_tableau_reach; a default depth is then min(32, 64 / reach)
 * steps, default sites_per_lane 8 up to 4 stages and 4 beyond. Until
 * a tableau is set, chain_rk4_step returns CHAIN_EINVAL. CHAIN_EINVAL also
 * for a handle of another scheme.
 */
int chain_rk4_set_tableau(chain_rk4 *h, const chain_rk4_tableau *t);

/*
 * Sites per side that one step of the tableau's method carries a change of
 * the state for the given model (the overlap per step of Sec. 2.3, exact for
 * the tableau's zero pattern): for dq/dt = p, dp/dt = F(q) with F reaching
 * R sites (R = 1, or 2 for the NNN models), stage argument Q_j reaches as far
 * as the momenta P_m it combines (a[j][m] != 0), P_j as far as the forces
 * F(Q_m) plus R, and the step as far as the stages with b[m] != 0. Classical
 * RK4: 2 (4 for NNN). Returns -1 for an invalid tableau or model (the
 * Roessler chain is not covered). No GPU is needed.
 */
int64_t chain_rk4_tableau_reach(int32_t model, const chain_rk4_tableau *t);

/*
 * Synchronise the handle's stream and report failures of its step calls
 * that the launch could not return: CHAIN_ETIMEOUT if, since the last check,
 * a step call with CHAIN_FLAG_EXCHANGE had a cluster give up waiting for its
 * neighbours (its results are then invalid; the kernel still finished).
 * Handles without that flag only synchronise.
 */
int chain_rk4_check(chain_rk4 *h);

/* Release a handle (host memory and cached graphs only). NULL is a no-op. */
int chain_rk4_destroy(chain_rk4 *h);

/* Static description of a status code; never NULL. */
const char *chain_rk4_strerror(int status);

/* Message of the last failure on the calling thread ("" if none). */
const char *chain_rk4_last_error(void);

/*
 * Batches: many independent chains advanced by ONE persistent launch.
 *
 * The launch holds as many workgroups as the device keeps resident. They
 * claim work items in a fixed order from a device counter: with
 * CHAIN_BATCH_RESIDENT_RINGS, first one item per short ring (n <= 1024), which
 * stays on chip for all of its steps; then, pass by pass, the cluster items,
 * each cluster pass the same as the fused method's (2*kdepth sites, rounded
 * up to 4, recomputed per side, Sec. 2.3). A chain is cut into wide clusters
 * of 64*sites_per_lane*4 sites (one workgroup of four wavefronts) followed by
 * at most three narrow clusters of 64*sites_per_lane sites (one wavefront),
 * whichever mix covers it in the fewest lane-sites; the last wide cluster of a
 * chain would otherwise keep only its remainder, and a short chain would fill
 * a quarter of a wide cluster. An item is one wide cluster or a pack of up to
 * four narrow clusters. A cluster's pass e starts once its own cluster and its
 * two neighbours have finished pass e-1 (per-cluster progress flags), so
 * passes of different clusters and chains overlap. Every chain gives the same
 * bits as when stepped alone (any handle settings, any grid, either cut).
 *
 * All handles of a batch share one model (CHAIN_QUARTIC or CHAIN_HARMONIC)
 * and one precision, use CHAIN_FUSED with CHAIN_SCHEME_RK4 (a handle given a
 * Butcher tableau is rejected with CHAIN_EINVAL), appear once, and must stay
 * valid while the batch runs them; each chain keeps its own dt. Calls that
 * overlap on one batch's workspace race.
 *
 * A batch is an object rather than a stateless call over handles: its
 * workspace (progress flags, the work counter, the item tables), the pinned
 * host staging of those tables and the per-launch timeout words persist
 * across step calls, so a steady stream of launches (the rounds of a job
 * server) allocates nothing, and rebind swaps the chain set in place.
 */
enum chain_batch_flags {
    CHAIN_BATCH_FENCES = 1,         /* hand cluster data between workgroups with
                                       ordinary loads and stores plus agent-scope
                                       cache write-back and invalidation, instead
                                       of device-coherent loads and stores */
    CHAIN_BATCH_RESIDENT_RINGS = 2, /* keep rings of at most 1024 sites on chip
                                       for all their steps (one item each, first);
                                       without it every chain is tiled, and the
                                       launch uses a kernel without the resident
                                       path (fewer registers, more wavefronts) */
    CHAIN_BATCH_WIDE_ONLY = 4       /* cut chains into wide clusters only (no
                                       narrow ones); the same results */
};

typedef struct chain_rk4_batch_desc {
    int64_t max_steps;       /* largest per-chain step count of one step call */
    int64_t max_clusters;    /* capacity for chain_rk4_batch_rebind: clusters
                                over all tiled chains (0 = what `hs` needs) */
    int32_t sites_per_lane;  /* 0 = default (8), else 4, 8 or 16 */
    int32_t kdepth;          /* steps per pass, 0 = default (32), else 2..32 */
    int32_t grid_blocks;     /* workgroups, 0 = as many as the device holds at
                                once; any value >= 1 gives the same results */
    int32_t flags;           /* 0, or CHAIN_BATCH_* flags OR-ed */
    int32_t spin_limit;      /* polls before a wait for a neighbour gives up,
                                0 = default (about 4 s); small values force
                                CHAIN_ETIMEOUT for failure-path tests */
    int32_t max_chains;      /* capacity for chain_rk4_batch_rebind: chains
                                (0 = count) */
} chain_rk4_batch_desc;

typedef struct chain_rk4_batch_plan {
    int32_t sites_per_lane, kdepth, waves_per_cluster, grid_blocks;
    int64_t halo;            /* recomputed sites per cluster side: 2 * kdepth
                                rounded up to a multiple of 4 (tiles start at
                                multiples of 4 sites, so every cluster starts
                                on a 16-byte boundary) */
    int64_t tile_max;        /* most sites a wide cluster keeps per pass */
    int64_t total_clusters;  /* clusters over all tiled chains */
    int64_t resident_chains; /* chains kept on chip for a whole launch */
    int64_t tile_narrow;     /* most sites a narrow cluster keeps per pass; 0 if
                                the shape has no narrow clusters (a one-wavefront
                                cluster must keep at least `halo` sites after its
                                two halos, or with CHAIN_BATCH_WIDE_ONLY) */
    int64_t narrow_clusters; /* of total_clusters, the narrow ones */
} chain_rk4_batch_plan;

/* Device workspace bytes (256-byte aligned) of a batch over hs[0..count):
 * per-cluster progress flags, the work counter, the item tables. 0 if the
 * arguments are invalid. */
size_t chain_rk4_batch_workspace_bytes(chain_rk4 *const *hs, int count,
                                       const chain_rk4_batch_desc *d);

/* Create a batch (host object plus a pinned host staging buffer for the
 * tables). `stream` carries every launch of the batch. */
int chain_rk4_batch_create(chain_rk4 *const *hs, int count, const chain_rk4_batch_desc *d,
                           void *workspace, size_t ws_bytes, void *stream,
                           chain_rk4_batch **out);

/*
 * Point an existing batch at another set of handles (same model and
 * precision; count <= max_chains; their clusters <= max_clusters), reusing
 * its workspace. Launches already enqueued keep the old set. Returns
 * CHAIN_ENOMEM if the set exceeds the capacity.
 */
int chain_rk4_batch_rebind(chain_rk4_batch *b, chain_rk4 *const *hs, int count);

/* The shape a batch with descriptor `d` would use (sites_per_lane, kdepth,
 * waves_per_cluster, halo, tile_max, tile_narrow; grid_blocks as given, 0 = as
 * many as the device holds; the cluster counts are 0), without a GPU or
 * handles.
 * CHAIN_EINVAL for a descriptor chain_rk4_batch_create would reject. */
int chain_rk4_batch_plan_for(const chain_rk4_batch_desc *d, chain_rk4_batch_plan *out);

/* Clusters a chain of n sites occupies in a batch of the given shape
 * (sites_per_lane and kdepth as in the descriptor, 0 = default) when it is
 * tiled, wide and narrow ones (the cut without narrow clusters never has
 * more); a ring kept on chip (CHAIN_BATCH_RESIDENT_RINGS) takes none. 0 for
 * invalid arguments. Used to size max_clusters. */
int64_t chain_rk4_batch_clusters(int64_t n, int32_t sites_per_lane, int32_t kdepth);

/*
 * How a tiled chain of n sites is cut in a batch with descriptor `d` (only
 * sites_per_lane, kdepth and flags are read): cluster i keeps the sites
 * [start[i], start[i] + keep[i]) and spans waves[i] wavefronts (4: wide, 1:
 * narrow). Fills the first min(count, cap) entries of the three arrays (host
 * memory, owned by the caller; NULL allowed when cap is 0) and returns count,
 * the number of clusters, or -1 with the last error set for invalid
 * arguments. Every start is a multiple of 4, the kept ranges tile [0, n) in
 * order, and with two or more clusters each keeps at least `halo` sites (its
 * neighbours' halos then lie in the adjacent clusters only).
 */
int64_t chain_rk4_batch_layout(int64_t n, const chain_rk4_batch_desc *d, int64_t *start,
                               int64_t *keep, int32_t *waves, int64_t cap);

/* Advance chain j by nsteps[j] (0..max_steps) steps in one persistent launch
 * (asynchronous; nsteps is read before the call returns). */
int chain_rk4_batch_step(chain_rk4_batch *b, const int64_t *nsteps);

/* Synchronise the batch's stream; CHAIN_ETIMEOUT if, in any launch since the
 * last chain_rk4_batch_check, a wait for a neighbour expired (the results of
 * that launch are then invalid; the kernel still terminated). */
int chain_rk4_batch_check(chain_rk4_batch *b);

/* Id of the last launch chain_rk4_batch_step enqueued (launches are numbered
 * 0, 1, ... per batch; a step call with every count 0 launches nothing), or
 * -1 if there was none. */
int chain_rk4_batch_last_launch(const chain_rk4_batch *b, int64_t *id);

/* Wait for launch `id` alone (not for launches enqueued after it) and return
 * CHAIN_ETIMEOUT if one of its waits for a neighbour expired, else CHAIN_OK.
 * Each launch's timeout word is copied to pinned host memory behind it, so
 * pipelined callers can check round R while round R+1 runs. CHAIN_EINVAL if
 * `id` was not enqueued or is older than the last 64 launches (their
 * timeouts are still reported by chain_rk4_batch_check). */
int chain_rk4_batch_check_launch(chain_rk4_batch *b, int64_t id);

/* Energies of every chain into e_out[count] (host), as chain_rk4_energy. */
int chain_rk4_batch_energy(chain_rk4_batch *b, double *e_out);

/* Report the shape the batch uses. */
int chain_rk4_batch_get_plan(const chain_rk4_batch *b, chain_rk4_batch_plan *out);

/* Release a batch (host memory only; waits for its last table upload).
 * NULL is a no-op. */
int chain_rk4_batch_destroy(chain_rk4_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* CHAIN_RK4_H */
