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

constexpr int kDefaultBatchSites = 4;
constexpr int kDefaultBatchDepth = 32;  // fastest of 16 and 32 on the 4096-chain batch
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

// Clusters of a tiled chain: keep at most `tile_max` sites each, in 4-site
// units split as evenly as possible.
void split_clusters(int64_t n, int64_t tile_max, int64_t *clusters, int64_t *uq, int64_t *ur) {
    int64_t G = (n + (tile_max - 4) - 1) / (tile_max - 4);
    if (G < 1) G = 1;
    const int64_t units = n / 4;
    *clusters = G;
    *uq = units / G;
    *ur = units % G;
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
    bool resident_rings = false;   // CHAIN_BATCH_RESIDENT_RINGS
};

int make_shape(int32_t sites_per_lane, int32_t kdepth, Shape *out) {
    if (sites_per_lane != 0 && sites_per_lane != 4 && sites_per_lane != 8 && sites_per_lane != 16)
        return fail(CHAIN_EINVAL, "sites_per_lane must be 0, 4, 8 or 16");
    if (kdepth != 0 && (kdepth < 2 || kdepth > 32))
        return fail(CHAIN_EINVAL, "batch kdepth must be 0 or 2..32");
    Shape sh;
    sh.sites = sites_per_lane ? sites_per_lane : kDefaultBatchSites;
    sh.depth = kdepth ? kdepth : kDefaultBatchDepth;
    const int64_t E = 64 * static_cast<int64_t>(sh.sites) * kBatchWaves;
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
    *out = sh;
    return CHAIN_OK;
}

int64_t clusters_of(int64_t n, const Shape &sh) {
    if (sh.resident_rings && n <= kBatchResidentSites) return 0;
    int64_t G, uq, ur;
    split_clusters(n, sh.tile_max, &G, &uq, &ur);
    return G;
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
    if ((d->flags & ~(CHAIN_BATCH_FENCES | CHAIN_BATCH_RESIDENT_RINGS)) != 0)
        return fail(CHAIN_EINVAL, "unknown batch flags");
    if (d->spin_limit < 0) return fail(CHAIN_EINVAL, "spin_limit must be >= 0");
    if (d->max_chains < 0 || d->max_clusters < 0)
        return fail(CHAIN_EINVAL, "max_chains and max_clusters must be >= 0");
    int rc = make_shape(d->sites_per_lane, d->kdepth, sh);
    sh->resident_rings = (d->flags & CHAIN_BATCH_RESIDENT_RINGS) != 0;
    return rc;
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
    L.item_chain = take(sizeof(int32_t) * nc);
    L.item_cluster = take(sizeof(int32_t) * nc);
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
    std::vector<int64_t> clusters, uq, ur;
    int64_t total_clusters = 0;
};

namespace {

void bind(chain_rk4_batch *b, chain_rk4 *const *hs, int count) {
    b->hs.assign(hs, hs + count);
    b->resident.assign(count, 0);
    b->clusters.assign(count, 0);
    b->uq.assign(count, 0);
    b->ur.assign(count, 0);
    b->total_clusters = 0;
    for (int i = 0; i < count; ++i) {
        const int64_t n = hs[i]->d.n;
        if (b->sh.resident_rings && n <= kBatchResidentSites) {
            b->resident[i] = 1;
            continue;
        }
        split_clusters(n, b->sh.tile_max, &b->clusters[i], &b->uq[i], &b->ur[i]);
        b->total_clusters += b->clusters[i];
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
    *out = P;
    return CHAIN_OK;
}

int64_t chain_rk4_batch_clusters(int64_t n, int32_t sites_per_lane, int32_t kdepth) {
    Shape sh;
    if (n < 1 || make_shape(sites_per_lane, kdepth, &sh) != CHAIN_OK) return 0;
    return clusters_of(n, sh);
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

    int64_t w = 0, flag = 0, slot = 0;
    for (int64_t i : tiled) {
        chain_rk4 *h = b->hs[i];
        BatchChain c{};
        c.front = h->front;
        c.back = h->back;
        c.n = h->d.n;
        c.dt = h->d.dt;
        c.uq = b->uq[i];
        c.ur = b->ur[i];
        c.clusters = static_cast<int32_t>(b->clusters[i]);
        c.passes = static_cast<int32_t>(passes[i].count());
        c.nhead = passes[i].nhead;
        c.head0 = passes[i].head0;
        c.head1 = passes[i].head1;
        c.tail = passes[i].tail;
        c.flag_base = static_cast<int32_t>(flag);
        for (int64_t g = 0; g < b->clusters[i]; ++g) {
            item_chain[w] = static_cast<int32_t>(slot);
            item_cluster[w] = static_cast<int32_t>(g);
            ++w;
        }
        flag += b->clusters[i];
        chains[slot++] = c;
    }
    const int64_t n_tiled = slot;
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
    // pass_off[e]: items before pass e (a pass holds the clusters of the
    // chains with more than e passes, a prefix of the ordered list)
    const int64_t max_p = tiled.empty() ? 0 : passes[tiled[0]].count();
    pass_off[0] = 0;
    {
        int64_t active = n_tiled, acc = 0;
        std::vector<int64_t> prefix(n_tiled + 1, 0);
        for (int64_t k = 0; k < n_tiled; ++k) prefix[k + 1] = prefix[k] + chains[k].clusters;
        for (int64_t e = 0; e < max_p; ++e) {
            while (active > 0 && chains[active - 1].passes <= e) --active;
            acc += prefix[active];
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
    P.total_clusters = b->total_clusters;
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
