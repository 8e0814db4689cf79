// batch.cpp -- host side of the batch calls in include/chain_rk4.h: builds the
// work-item tables of a persistent launch over many chains and enqueues it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "chain_rk4.h"
#include "handle.hpp"
#include "launch.hpp"

using namespace chainrk4;

namespace {

constexpr size_t kAlign = 256;
size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// The fastest shape on the 4096-chain batch (2000 steps): S=8 k=32, where
// chain remainders take one-wavefront clusters (6.55 against 6.11e11 SU/s
// for S=4 in FP64, 9.23 against 8.83e11 with FP32 and compensated update).
constexpr int kDefaultBatchSites = 8;
constexpr int kDefaultBatchDepth = 32;
constexpr int kSpinLimit = 1 << 22;  // polls (each with a short sleep) before a wait gives up
// Launches whose timeout word stays readable one by one (a ring of pinned
// host words, each filled by a copy queued behind its launch).
constexpr int64_t kLaunchRing = 64;

// Per-chain pass list of a launch: `head` passes first (0 or 2 entries), then
// `mid` full passes of `depth` steps, then an optional `tail` pass. The pass
// count is even whenever a pass of two or more steps exists to split, so the
// state ends in the caller's buffers.
struct PassList {
    int32_t nhead = 0, head0 = 0, head1 = 0;
    int64_t mid = 0;
    int32_t tail = 0;
    int64_t count() const { return nhead + mid + (tail ? 1 : 0); }
};

PassList make_passes(int64_t nsteps, int depth) {
    PassList L;
    L.mid = nsteps / depth;
    L.tail = static_cast<int32_t>(nsteps % depth);
    if (L.count() % 2 == 1) {
        if (L.mid > 0 && depth >= 2) {  // split the first full pass
            L.mid -= 1;
            L.nhead = 2;
            L.head0 = depth / 2;
            L.head1 = depth - depth / 2;
        } else if (L.mid == 0 && L.tail >= 2) {  // a single short pass: split it
            L.nhead = 2;
            L.head0 = L.tail / 2;
            L.head1 = L.tail - L.tail / 2;
            L.tail = 0;
        }
    }
    return L;
}

struct Layout {
    size_t flags, counter, error, zero_bytes;  // zeroed before each launch
    size_t chains, item_chain, item_cluster, pass_off, table_bytes;
    size_t total;
};

// Cluster shape of a batch: sites per lane, pass depth, halo, kept sites.
struct Shape {
    int sites = 0, depth = 0;
    int64_t halo = 0, tile_max = 0;
    int64_t tile_narrow = 0;       // 0: no narrow clusters
    bool resident_rings = false;   // CHAIN_BATCH_RESIDENT_RINGS
};

int make_shape(int32_t sites_per_lane, int32_t kdepth, int32_t flags, Shape *out) {
    if (sites_per_lane != 0 && sites_per_lane != 4 && sites_per_lane != 8 && sites_per_lane != 16)
        return fail(CHAIN_EINVAL, "sites_per_lane must be 0, 4, 8 or 16");
    if (kdepth != 0 && (kdepth < 2 || kdepth > 32))
        return fail(CHAIN_EINVAL, "batch kdepth must be 0 or 2..32");
    Shape sh;
    sh.sites = sites_per_lane ? sites_per_lane : kDefaultBatchSites;
    sh.depth = kdepth ? kdepth : kDefaultBatchDepth;
    const int64_t E = 64 * static_cast<int64_t>(sh.sites) * kBatchWaves;
    const int64_t E1 = 64 * static_cast<int64_t>(sh.sites);
    // A step's wrong edge values travel 2 sites into a cluster of the
    // quartic or harmonic chain (dq/dt = p is local), so the halo covers
    // 2*depth sites, rounded up to 4: cluster tiles start at multiples of 4
    // sites, so every cluster origin then sits on a 16-byte boundary of the
    // FP64 and FP32 state arrays (the lanes' vector accesses need it; a wider
    // overlap keeps the kept sites exact, Sec. 2.3). Every cluster keeps at
    // least `halo` sites (so only neighbouring clusters overlap), with room to
    // spare for the 4-site rounding.
    auto halo_of = [](int depth) { return (2 * static_cast<int64_t>(depth) + 3) / 4 * 4; };
    while (E < 4 * halo_of(sh.depth) + 16 && sh.depth > 2) --sh.depth;
    sh.halo = halo_of(sh.depth);
    sh.tile_max = E - 2 * sh.halo;
    if (!(flags & CHAIN_BATCH_WIDE_ONLY) && E1 >= 4 * sh.halo + 16) sh.tile_narrow = E1 - 2 * sh.halo;
    sh.resident_rings = (flags & CHAIN_BATCH_RESIDENT_RINGS) != 0;
    *out = sh;
    return CHAIN_OK;
}

// How a tiled chain is cut: `wide` clusters keeping 4*(uq + (i < ur)) sites,
// then `narrow` ones keeping 4*(nuq + (j < nur)); the last cluster also keeps
// the n % 4 remainder.
struct Cut {
    int64_t wide = 0, narrow = 0, uq = 0, ur = 0, nuq = 0, nur = 0;
    int64_t clusters() const { return wide + narrow; }
};

// The cut of n sites in the fewest lane-sites (ties: fewer clusters). A
// cluster holds at most cap = tile/4 - 1 units of 4 sites (room for the
// remainder) and, when the chain has two or more clusters, at least halo/4
// (each neighbour's halo then lies in the adjacent cluster). Four narrow
// clusters cost one wide one and hold less, so at most three are used.
Cut cut_chain(int64_t n, const Shape &sh) {
    const int64_t E4 = 64 * static_cast<int64_t>(sh.sites) * kBatchWaves;
    const int64_t E1 = 64 * static_cast<int64_t>(sh.sites);
    const int64_t U = n / 4, c4 = sh.tile_max / 4 - 1, m = sh.halo / 4;
    const int64_t c1 = sh.tile_narrow ? sh.tile_narrow / 4 - 1 : 0;
    Cut best;
    int64_t best_cost = -1;
    for (int64_t g1 = 0; g1 <= (sh.tile_narrow ? kMaxNarrow : 0); ++g1) {
        int64_t g4 = U > g1 * c1 ? (U - g1 * c1 + c4 - 1) / c4 : 0;
        if (g4 + g1 == 0) g4 = 1;  // n < 4: one wide cluster
        const int64_t G = g4 + g1;
        if (G >= 2 && U < G * m) continue;
        const int64_t cost = g4 * E4 + g1 * E1;
        if (best_cost >= 0 && (cost > best_cost || (cost == best_cost && G >= best.clusters())))
            continue;
        // narrow clusters take what the wide ones cannot hold, but at least
        // the minimum each; with G >= 2 the wide ones then keep >= m each
        const int64_t u1 = g1 ? std::max(g1 * m, U - g4 * c4) : 0;
        const int64_t u4 = U - u1;
        Cut c;
        c.wide = g4;
        c.narrow = g1;
        if (g4) {
            c.uq = u4 / g4;
            c.ur = u4 % g4;
        }
        if (g1) {
            c.nuq = u1 / g1;
            c.nur = u1 % g1;
        }
        best = c;
        best_cost = cost;
    }
    return best;
}

// Kept range of cluster i of a cut (the same arithmetic as the kernel's).
void cluster_span(const Cut &c, int64_t n, int64_t i, int64_t *start, int64_t *keep) {
    int64_t units;
    if (i < c.wide) {
        *start = 4 * (i * c.uq + std::min(i, c.ur));
        units = c.uq + (i < c.ur ? 1 : 0);
    } else {
        const int64_t j = i - c.wide;
        *start = 4 * (c.wide * c.uq + c.ur + j * c.nuq + std::min(j, c.nur));
        units = c.nuq + (j < c.nur ? 1 : 0);
    }
    *keep = (i == c.clusters() - 1) ? n - *start : 4 * units;
}

int64_t clusters_of(int64_t n, const Shape &sh) {
    if (sh.resident_rings && n <= kBatchResidentSites) return 0;
    return cut_chain(n, sh).clusters();
}

// Validate a handle set against a batch's model and precision.
int check_handles(chain_rk4 *const *hs, int count, int model, int prec) {
    if (!hs || count < 1) return fail(CHAIN_EINVAL, "a batch needs count >= 1 handles");
    for (int i = 0; i < count; ++i) {
        if (!hs[i]) return fail(CHAIN_EINVAL, "handle %d is NULL", i);
        if (hs[i]->d.method != CHAIN_FUSED)
            return fail(CHAIN_EINVAL, "handle %d does not use the fused method", i);
        if (hs[i]->d.scheme != CHAIN_SCHEME_RK4)
            return fail(CHAIN_EINVAL, "handle %d: batches run classical RK4 only (no tableau)", i);
        if (hs[i]->d.model != model || hs[i]->d.prec != prec)
            return fail(CHAIN_EINVAL, "handle %d differs in model or precision", i);
        if (hs[i]->d.model != CHAIN_QUARTIC && hs[i]->d.model != CHAIN_HARMONIC)
            return fail(CHAIN_EINVAL, "handle %d: batches take the quartic and harmonic models only", i);
        if (hs[i]->d.prec == CHAIN_FP32_KAHAN64 || hs[i]->d.prec == CHAIN_FP32)
            return fail(CHAIN_EINVAL, "handle %d: batches take CHAIN_FP64 or CHAIN_FP32_KAHAN", i);
    }
    std::vector<chain_rk4 *> sorted(hs, hs + count);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return fail(CHAIN_EINVAL, "a handle appears twice");
    return CHAIN_OK;
}

int check_desc(const chain_rk4_batch_desc *d, Shape *sh) {
    if (!d) return fail(CHAIN_EINVAL, "batch descriptor is NULL");
    if (d->max_steps < 0) return fail(CHAIN_EINVAL, "max_steps must be >= 0");
    if (d->grid_blocks < 0) return fail(CHAIN_EINVAL, "grid_blocks must be >= 0");
    if ((d->flags & ~(CHAIN_BATCH_FENCES | CHAIN_BATCH_RESIDENT_RINGS | CHAIN_BATCH_WIDE_ONLY)) != 0)
        return fail(CHAIN_EINVAL, "unknown batch flags");
    if (d->spin_limit < 0) return fail(CHAIN_EINVAL, "spin_limit must be >= 0");
    if (d->max_chains < 0 || d->max_clusters < 0)
        return fail(CHAIN_EINVAL, "max_chains and max_clusters must be >= 0");
    return make_shape(d->sites_per_lane, d->kdepth, d->flags, sh);
}

Layout batch_layout(int64_t chains, int64_t clusters, int64_t max_passes) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += round_up(b);
        return o;
    };
    const size_t nc = static_cast<size_t>(std::max<int64_t>(clusters, 1));
    L.flags = take(sizeof(int32_t) * nc);
    L.counter = take(sizeof(unsigned long long));
    L.error = take(sizeof(int32_t));
    L.zero_bytes = off;
    const size_t t0 = off;
    L.chains = take(sizeof(BatchChain) * static_cast<size_t>(chains));
    // at most one item per cluster, kBatchWaves slots each
    L.item_chain = take(sizeof(int32_t) * kBatchWaves * nc);
    L.item_cluster = take(sizeof(int32_t) * kBatchWaves * nc);
    L.pass_off = take(sizeof(int64_t) * static_cast<size_t>(max_passes + 2));
    L.table_bytes = off - t0;
    L.total = off;
    return L;
}

// Capacity a descriptor asks for, given the first handle set.
void capacity(chain_rk4 *const *hs, int count, const chain_rk4_batch_desc *d, const Shape &sh,
              int64_t *chains, int64_t *clusters, int64_t *passes) {
    int64_t need = 0;
    for (int i = 0; i < count; ++i) need += clusters_of(hs[i]->d.n, sh);
    *chains = std::max<int64_t>(count, d->max_chains);
    *clusters = std::max<int64_t>(need, d->max_clusters);
    *passes = make_passes(d->max_steps, sh.depth).count() + 1;
}

}  // namespace

struct chain_rk4_batch {
    std::vector<chain_rk4 *> hs;
    chain_rk4_batch_desc d{};
    int model = 0, prec = 0;
    Shape sh;
    int64_t cap_chains = 0, cap_clusters = 0, max_passes = 0;
    char *ws = nullptr;
    Layout L{};
    hipStream_t stream = nullptr;
    void *staging = nullptr;       // pinned host copy of the tables
    hipEvent_t staged = nullptr;   // the last table upload has been read
    bool staged_pending = false;
    // timeout word of each of the last kLaunchRing launches (pinned), and an
    // event behind the copy of each
    int32_t *launch_err = nullptr;
    hipEvent_t launch_done[kLaunchRing] = {};
    int64_t launches = 0;          // launches enqueued so far (ids 0..launches-1)
    int64_t folded = 0;            // launches whose word is in pending_error
    bool pending_error = false;    // a launch since the last check timed out
    // per chain of the current set
    std::vector<char> resident;
    std::vector<Cut> cuts;
    int64_t total_clusters = 0, narrow_clusters = 0;
};

namespace {

void bind(chain_rk4_batch *b, chain_rk4 *const *hs, int count) {
    b->hs.assign(hs, hs + count);
    b->resident.assign(count, 0);
    b->cuts.assign(count, Cut{});
    b->total_clusters = 0;
    b->narrow_clusters = 0;
    for (int i = 0; i < count; ++i) {
        const int64_t n = hs[i]->d.n;
        if (b->sh.resident_rings && n <= kBatchResidentSites) {
            b->resident[i] = 1;
            continue;
        }
        b->cuts[i] = cut_chain(n, b->sh);
        b->total_clusters += b->cuts[i].clusters();
        b->narrow_clusters += b->cuts[i].narrow;
    }
}

// Fold the timeout words of launches [folded, upto) into pending_error;
// those launches must have completed.
void fold_through(chain_rk4_batch *b, int64_t upto) {
    for (; b->folded < upto; ++b->folded)
        if (__atomic_load_n(&b->launch_err[b->folded % kLaunchRing], __ATOMIC_ACQUIRE) != 0)
            b->pending_error = true;
}

bool has_resident_items(const chain_rk4_batch *b) {
    for (char r : b->resident)
        if (r) return true;
    return false;
}

}  // namespace

extern "C" {

int chain_rk4_batch_plan_for(const chain_rk4_batch_desc *d, chain_rk4_batch_plan *out) {
    if (!out) return fail(CHAIN_EINVAL, "out is NULL");
    Shape sh;
    int rc = check_desc(d, &sh);
    if (rc != CHAIN_OK) return rc;
    chain_rk4_batch_plan P{};
    P.sites_per_lane = sh.sites;
    P.kdepth = sh.depth;
    P.waves_per_cluster = kBatchWaves;
    P.grid_blocks = d->grid_blocks;
    P.halo = sh.halo;
    P.tile_max = sh.tile_max;
    P.tile_narrow = sh.tile_narrow;
    *out = P;
    return CHAIN_OK;
}

int64_t chain_rk4_batch_clusters(int64_t n, int32_t sites_per_lane, int32_t kdepth) {
    Shape sh;
    if (n < 1 || make_shape(sites_per_lane, kdepth, 0, &sh) != CHAIN_OK) return 0;
    return clusters_of(n, sh);
}

int64_t chain_rk4_batch_layout(int64_t n, const chain_rk4_batch_desc *d, int64_t *start,
                               int64_t *keep, int32_t *waves, int64_t cap) {
    if (!d) {
        fail(CHAIN_EINVAL, "batch descriptor is NULL");
        return -1;
    }
    if (n < 1) {
        fail(CHAIN_EINVAL, "n must be >= 1");
        return -1;
    }
    if (cap < 0 || (cap > 0 && (!start || !keep || !waves))) {
        fail(CHAIN_EINVAL, "cap must be >= 0, and the arrays non-NULL when cap > 0");
        return -1;
    }
    Shape sh;
    if (make_shape(d->sites_per_lane, d->kdepth, d->flags, &sh) != CHAIN_OK) return -1;
    const Cut c = cut_chain(n, sh);
    for (int64_t i = 0; i < c.clusters() && i < cap; ++i) {
        cluster_span(c, n, i, &start[i], &keep[i]);
        waves[i] = i < c.wide ? kBatchWaves : 1;
    }
    return c.clusters();
}

size_t chain_rk4_batch_workspace_bytes(chain_rk4 *const *hs, int count,
                                       const chain_rk4_batch_desc *d) {
    Shape sh;
    if (check_desc(d, &sh) != CHAIN_OK) return 0;
    if (!hs || count < 1 || !hs[0]) return 0;
    if (check_handles(hs, count, hs[0]->d.model, hs[0]->d.prec) != CHAIN_OK) return 0;
    int64_t chains, clusters, passes;
    capacity(hs, count, d, sh, &chains, &clusters, &passes);
    return batch_layout(chains, clusters, passes).total;
}

int chain_rk4_batch_create(chain_rk4 *const *hs, int count, const chain_rk4_batch_desc *d,
                           void *workspace, size_t ws_bytes, void *stream, chain_rk4_batch **out) {
    if (!out) return fail(CHAIN_EINVAL, "out is NULL");
    *out = nullptr;
    Shape sh;
    int rc = check_desc(d, &sh);
    if (rc != CHAIN_OK) return rc;
    if (!hs || count < 1 || !hs[0]) return fail(CHAIN_EINVAL, "a batch needs count >= 1 handles");
    rc = check_handles(hs, count, hs[0]->d.model, hs[0]->d.prec);
    if (rc != CHAIN_OK) return rc;
    int64_t chains, clusters, passes;
    capacity(hs, count, d, sh, &chains, &clusters, &passes);
    const Layout L = batch_layout(chains, clusters, passes);
    if (ws_bytes < L.total)
        return fail(CHAIN_ENOMEM, "batch workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)))
        return fail(CHAIN_EINVAL, "batch workspace must be non-NULL and 256-byte aligned");
    chain_rk4_batch *b = new (std::nothrow) chain_rk4_batch();
    if (!b) return fail(CHAIN_ENOMEM, "out of host memory");
    b->d = *d;
    b->model = hs[0]->d.model;
    b->prec = hs[0]->d.prec;
    b->sh = sh;
    b->cap_chains = chains;
    b->cap_clusters = clusters;
    b->max_passes = passes;
    b->L = L;
    b->ws = static_cast<char *>(workspace);
    b->stream = static_cast<hipStream_t>(stream);
    bind(b, hs, count);
    hipError_t e = hipHostMalloc(&b->staging, b->L.table_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&b->launch_err), sizeof(int32_t) * kLaunchRing,
                          hipHostMallocDefault);
    for (int64_t i = 0; e == hipSuccess && i < kLaunchRing; ++i)
        e = hipEventCreateWithFlags(&b->launch_done[i], hipEventDisableTiming);
    if (e != hipSuccess) {
        chain_rk4_batch_destroy(b);
        return hip_fail(e, "batch staging buffer");
    }
    *out = b;
    return CHAIN_OK;
}

int chain_rk4_batch_rebind(chain_rk4_batch *b, chain_rk4 *const *hs, int count) {
    if (!b) return fail(CHAIN_EINVAL, "batch is NULL");
    int rc = check_handles(hs, count, b->model, b->prec);
    if (rc != CHAIN_OK) return rc;
    if (count > b->cap_chains)
        return fail(CHAIN_ENOMEM, "%d chains exceed the batch capacity of %lld", count,
                    (long long)b->cap_chains);
    int64_t need = 0;
    for (int i = 0; i < count; ++i) need += clusters_of(hs[i]->d.n, b->sh);
    if (need > b->cap_clusters)
        return fail(CHAIN_ENOMEM, "%lld clusters exceed the batch capacity of %lld",
                    (long long)need, (long long)b->cap_clusters);
    bind(b, hs, count);
    return CHAIN_OK;
}

int chain_rk4_batch_step(chain_rk4_batch *b, const int64_t *nsteps) {
    if (!b || !nsteps) return fail(CHAIN_EINVAL, "batch and nsteps must be non-NULL");
    const int64_t count = static_cast<int64_t>(b->hs.size());
    for (int64_t i = 0; i < count; ++i)
        if (nsteps[i] < 0 || nsteps[i] > b->d.max_steps)
            return fail(CHAIN_EINVAL, "nsteps[%lld] = %lld outside 0..%lld", (long long)i,
                        (long long)nsteps[i], (long long)b->d.max_steps);

    // Tiled chains ordered by pass count (descending): the chains still
    // running at pass e are then a prefix, and the items of every pass are a
    // prefix of one (chain, cluster) table.
    std::vector<int64_t> tiled, res;
    std::vector<PassList> passes(count);
    for (int64_t i = 0; i < count; ++i) {
        if (nsteps[i] == 0) continue;
        if (b->resident[i]) {
            res.push_back(i);
        } else {
            passes[i] = make_passes(nsteps[i], b->sh.depth);
            tiled.push_back(i);
        }
    }
    std::stable_sort(tiled.begin(), tiled.end(), [&](int64_t x, int64_t y) {
        return passes[x].count() > passes[y].count();
    });
    if (tiled.empty() && res.empty()) return CHAIN_OK;

    if (b->staged_pending) {
        HIP_TRY(hipEventSynchronize(b->staged));
        b->staged_pending = false;
    }
    char *host = static_cast<char *>(b->staging);
    const size_t t0 = b->L.chains;
    BatchChain *chains = reinterpret_cast<BatchChain *>(host + (b->L.chains - t0));
    int32_t *item_chain = reinterpret_cast<int32_t *>(host + (b->L.item_chain - t0));
    int32_t *item_cluster = reinterpret_cast<int32_t *>(host + (b->L.item_cluster - t0));
    int64_t *pass_off = reinterpret_cast<int64_t *>(host + (b->L.pass_off - t0));

    // Items in chain order: a chain's wide clusters, then its narrow ones
    // into the open pack (a pack opened by an earlier chain, else a new one
    // at this point). Every item's first chain is then no later than any
    // item after it, so the items whose first chain still runs at pass e
    // are a prefix of the table (first[k]: items before chain k's).
    int64_t w = 0, flag = 0, slot = 0;
    int64_t pack = -1, pack_used = 0;  // open pack: item index, slots taken
    std::vector<int64_t> first(tiled.size() + 1, 0);
    for (int64_t i : tiled) {
        chain_rk4 *h = b->hs[i];
        const Cut &cut = b->cuts[i];
        BatchChain c{};
        c.front = h->front;
        c.back = h->back;
        c.n = h->d.n;
        c.dt = h->d.dt;
        c.uq = cut.uq;
        c.ur = cut.ur;
        c.wide = static_cast<int32_t>(cut.wide);
        c.nuq = static_cast<int32_t>(cut.nuq);
        c.nur = static_cast<int32_t>(cut.nur);
        c.clusters = static_cast<int32_t>(cut.clusters());
        c.passes = static_cast<int32_t>(passes[i].count());
        c.nhead = passes[i].nhead;
        c.head0 = passes[i].head0;
        c.head1 = passes[i].head1;
        c.tail = passes[i].tail;
        c.flag_base = static_cast<int32_t>(flag);
        first[slot] = w;
        for (int64_t g = 0; g < cut.wide; ++g) {
            item_chain[kBatchWaves * w] = static_cast<int32_t>(slot);
            item_cluster[kBatchWaves * w] = static_cast<int32_t>(g);
            item_chain[kBatchWaves * w + 1] = kWideItem;
            ++w;
        }
        for (int64_t g = cut.wide; g < cut.clusters(); ++g) {
            if (pack < 0 || pack_used == kBatchWaves) {
                pack = w++;
                pack_used = 0;
                for (int v = 0; v < kBatchWaves; ++v) {
                    item_chain[kBatchWaves * pack + v] = kEmptySlot;
                    item_cluster[kBatchWaves * pack + v] = 0;
                }
            }
            item_chain[kBatchWaves * pack + pack_used] = static_cast<int32_t>(slot);
            item_cluster[kBatchWaves * pack + pack_used] = static_cast<int32_t>(g);
            ++pack_used;
        }
        flag += cut.clusters();
        chains[slot++] = c;
    }
    const int64_t n_tiled = slot;
    first[n_tiled] = w;
    for (int64_t i : res) {
        chain_rk4 *h = b->hs[i];
        BatchChain c{};
        c.front = h->front;
        c.back = h->back;
        c.n = h->d.n;
        c.dt = h->d.dt;
        c.nsteps = nsteps[i];
        chains[slot++] = c;
    }
    // pass_off[e]: items before pass e. Pass e holds the items whose first
    // chain has more than e passes (chains are ordered by pass count); a
    // pack slot whose chain has no pass e left is skipped by its wavefront.
    const int64_t max_p = tiled.empty() ? 0 : passes[tiled[0]].count();
    pass_off[0] = 0;
    {
        int64_t active = n_tiled, acc = 0;
        for (int64_t e = 0; e < max_p; ++e) {
            while (active > 0 && chains[active - 1].passes <= e) --active;
            acc += first[active];
            pass_off[e + 1] = acc;
        }
        pass_off[max_p + 1] = acc + 1;  // sentinel for the forward scan
    }
    const int64_t total_items = static_cast<int64_t>(res.size()) + pass_off[max_p];

    BatchArgs a{};
    a.chains = reinterpret_cast<const BatchChain *>(b->ws + b->L.chains);
    a.pass_off = reinterpret_cast<const int64_t *>(b->ws + b->L.pass_off);
    a.item_chain = reinterpret_cast<const int32_t *>(b->ws + b->L.item_chain);
    a.item_cluster = reinterpret_cast<const int32_t *>(b->ws + b->L.item_cluster);
    a.flags = reinterpret_cast<int32_t *>(b->ws + b->L.flags);
    a.counter = reinterpret_cast<unsigned long long *>(b->ws + b->L.counter);
    a.error = reinterpret_cast<int32_t *>(b->ws + b->L.error);
    a.total_items = total_items;
    a.halo = b->sh.halo;
    a.n_resident = static_cast<int32_t>(res.size());
    a.n_tiled = static_cast<int32_t>(n_tiled);
    a.max_passes = static_cast<int32_t>(max_p);
    a.depth = b->sh.depth;
    a.spin_limit = b->d.spin_limit ? b->d.spin_limit : kSpinLimit;
    a.fences = (b->d.flags & CHAIN_BATCH_FENCES) ? 1 : 0;

    int blocks = b->d.grid_blocks;
    if (blocks == 0) {
        blocks = persistent_capacity(b->model, b->prec, b->sh.sites, has_resident_items(b));
        if (blocks <= 0) return fail(CHAIN_EHIP, "occupancy query failed");
    }
    if (blocks > total_items) blocks = static_cast<int>(total_items);

    hipError_t e = launch_fill_zero(b->ws, b->L.zero_bytes, b->stream);
    if (e != hipSuccess) return hip_fail(e, "clearing batch flags");
    HIP_TRY(hipMemcpyAsync(b->ws + b->L.chains, b->staging, b->L.table_bytes, hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipEventRecord(b->staged, b->stream));
    b->staged_pending = true;
    e = launch_persistent(b->model, b->prec, b->sh.sites, blocks, a, b->stream);
    if (e != hipSuccess) return hip_fail(e, "persistent launch");
    // a tiled chain with a single one-step pass ends in its back buffer
    for (int64_t i : tiled) {
        if (passes[i].count() % 2 == 1) {
            chain_rk4 *h = b->hs[i];
            const size_t bytes = static_cast<size_t>(h->d.n) * elem_bytes(h->d.prec);
            HIP_TRY(hipMemcpyAsync(h->front.q, h->back.q, bytes, hipMemcpyDeviceToDevice, b->stream));
            HIP_TRY(hipMemcpyAsync(h->front.p, h->back.p, bytes, hipMemcpyDeviceToDevice, b->stream));
            if (has_carries(h->d.prec)) {
                const size_t cb = static_cast<size_t>(h->d.n) * carry_bytes(h->d.prec);
                HIP_TRY(hipMemcpyAsync(h->front.cq, h->back.cq, cb, hipMemcpyDeviceToDevice, b->stream));
                HIP_TRY(hipMemcpyAsync(h->front.cp, h->back.cp, cb, hipMemcpyDeviceToDevice, b->stream));
            }
        }
    }
    // this launch's timeout word into its ring slot; the launch that used the
    // slot before (kLaunchRing launches ago) is folded into the pending error
    // of chain_rk4_batch_check first
    const int64_t ring = b->launches % kLaunchRing;
    if (b->launches >= kLaunchRing) {
        HIP_TRY(hipEventSynchronize(b->launch_done[ring]));
        fold_through(b, b->launches - kLaunchRing + 1);
    }
    HIP_TRY(hipMemcpyAsync(&b->launch_err[ring], b->ws + b->L.error, sizeof(int32_t),
                           hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipEventRecord(b->launch_done[ring], b->stream));
    ++b->launches;
    return CHAIN_OK;
}

int chain_rk4_batch_last_launch(const chain_rk4_batch *b, int64_t *id) {
    if (!b || !id) return fail(CHAIN_EINVAL, "batch and id must be non-NULL");
    *id = b->launches - 1;
    return CHAIN_OK;
}

int chain_rk4_batch_check_launch(chain_rk4_batch *b, int64_t id) {
    if (!b) return fail(CHAIN_EINVAL, "batch is NULL");
    if (id < 0 || id >= b->launches)
        return fail(CHAIN_EINVAL, "launch %lld was not enqueued", (long long)id);
    if (id < b->launches - kLaunchRing)
        return fail(CHAIN_EINVAL, "launch %lld is older than the last %lld launches",
                    (long long)id, (long long)kLaunchRing);
    const int64_t slot = id % kLaunchRing;
    HIP_TRY(hipEventSynchronize(b->launch_done[slot]));
    if (__atomic_load_n(&b->launch_err[slot], __ATOMIC_ACQUIRE) != 0)
        return fail(CHAIN_ETIMEOUT, "launch %lld: a work item's wait for its neighbours timed out",
                    (long long)id);
    return CHAIN_OK;
}

int chain_rk4_batch_check(chain_rk4_batch *b) {
    if (!b) return fail(CHAIN_EINVAL, "batch is NULL");
    HIP_TRY(hipStreamSynchronize(b->stream));
    fold_through(b, b->launches);
    const bool err = b->pending_error;
    b->pending_error = false;
    if (err) return fail(CHAIN_ETIMEOUT, "a work item's wait for its neighbours timed out");
    return CHAIN_OK;
}

int chain_rk4_batch_energy(chain_rk4_batch *b, double *e_out) {
    if (!b || !e_out) return fail(CHAIN_EINVAL, "batch and e_out must be non-NULL");
    int status = CHAIN_OK;
    for (size_t i = 0; i < b->hs.size(); ++i) {
        chain_rk4 *h = b->hs[i];
        hipStream_t keep = h->stream;
        h->stream = b->stream;
        const int rc = chain_rk4_energy(h, &e_out[i]);
        h->stream = keep;
        if (rc == CHAIN_ENONFINITE) status = rc;
        else if (rc != CHAIN_OK) return rc;
    }
    return status;
}

int chain_rk4_batch_get_plan(const chain_rk4_batch *b, chain_rk4_batch_plan *out) {
    if (!b || !out) return fail(CHAIN_EINVAL, "batch and out must be non-NULL");
    chain_rk4_batch_plan P{};
    P.sites_per_lane = b->sh.sites;
    P.kdepth = b->sh.depth;
    P.waves_per_cluster = kBatchWaves;
    P.grid_blocks = b->d.grid_blocks ? b->d.grid_blocks
                                     : persistent_capacity(b->model, b->prec, b->sh.sites,
                                                           has_resident_items(b));
    P.halo = b->sh.halo;
    P.tile_max = b->sh.tile_max;
    P.tile_narrow = b->sh.tile_narrow;
    P.total_clusters = b->total_clusters;
    P.narrow_clusters = b->narrow_clusters;
    int64_t nres = 0;
    for (char r : b->resident) nres += r;
    P.resident_chains = nres;
    *out = P;
    return CHAIN_OK;
}

int chain_rk4_batch_destroy(chain_rk4_batch *b) {
    if (!b) return CHAIN_OK;
    if (b->staged) {
        if (b->staged_pending) (void)hipEventSynchronize(b->staged);
        (void)hipEventDestroy(b->staged);
    }
    if (b->staging) (void)hipHostFree(b->staging);
    // the copy of the last launch's timeout word (and, in stream order, every
    // earlier one) must land before its host word is freed
    if (b->launches > 0) (void)hipEventSynchronize(b->launch_done[(b->launches - 1) % kLaunchRing]);
    for (hipEvent_t ev : b->launch_done)
        if (ev) (void)hipEventDestroy(ev);
    if (b->launch_err) (void)hipHostFree(b->launch_err);
    delete b;
    return CHAIN_OK;
}

}  // extern "C"
