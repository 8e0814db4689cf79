// Drives the host-only paths of the C ABI (include/chain_rk4.h) under
// AddressSanitizer and UndefinedBehaviorSanitizer, with no GPU: the planners
// over every descriptor they accept or refuse, workspace sizes, the reach of
// random explicit tableaus, argument validation of every call that takes a
// handle or a batch, and the status strings. Built and run by
// tests/test_sanitizers.py; exits 0 when every invariant holds.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>

#include "chain_rk4.h"

static int failures = 0;

#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "FAIL line %d: %s\n", __LINE__, #cond);         \
            if (++failures > 20) return 1;                                       \
        }                                                                        \
    } while (0)

static chain_rk4_desc desc(int64_t n, int model, int prec, int s, int w, int k, int flags,
                           int scheme, int method = CHAIN_FUSED) {
    chain_rk4_desc d{};
    d.n = n;
    d.model = model;
    d.prec = prec;
    d.dt = 0.01;
    d.method = method;
    d.sites_per_lane = s;
    d.kdepth = k;
    d.waves_per_cluster = w;
    d.flags = flags;
    d.scheme = scheme;
    return d;
}

static chain_rk4_tableau random_tableau(std::mt19937_64 &rng, int stages) {
    std::uniform_real_distribution<double> u(-1.0, 1.0), z(0.0, 1.0);
    chain_rk4_tableau t{};
    t.stages = stages;
    for (int j = 0; j < stages; ++j) {
        for (int m = 0; m < j; ++m) t.a[j][m] = z(rng) < 0.4 ? 0.0 : u(rng);
        t.b[j] = z(rng) < 0.3 ? 0.0 : u(rng);
    }
    return t;
}

int main() {
    const int64_t lengths[] = {1, 2, 3, 100, 4096, 4097, (1 << 17) + 1, (1 << 21) + 1,
                               int64_t(1) << 24, int64_t(1) << 40, (int64_t(1) << 40) + 1, 0, -3};
    long accepted = 0, refused = 0;
    // every classical descriptor: plan_for and workspace_bytes agree on
    // validity; accepted plans are 16-byte aligned and keep sites
    for (int64_t n : lengths)
        for (int model = -1; model <= 5; ++model)
            for (int prec = -1; prec <= 4; ++prec)
                for (int s : {0, 1, 2, 4, 8, 16})
                    for (int w : {0, 1, 3, 4, 8})
                        for (int k : {-1, 0, 1, 3, 7, 16, 25, 32, 33})
                            for (int flags : {0, int(CHAIN_FLAG_GRAPH), int(CHAIN_FLAG_RESIDENT), 64})
                                for (int method : {int(CHAIN_FUSED), int(CHAIN_NAIVE)}) {
                                    chain_rk4_desc d = desc(n, model, prec, s, w, k, flags,
                                                            CHAIN_SCHEME_RK4, method);
                                    chain_rk4_plan P{};
                                    const int rc = chain_rk4_plan_for(&d, nullptr, &P);
                                    const size_t ws = chain_rk4_workspace_bytes(&d);
                                    CHECK((rc == CHAIN_OK) == (ws > 0));
                                    if (rc != CHAIN_OK) {
                                        CHECK(rc == CHAIN_EINVAL);
                                        CHECK(std::strlen(chain_rk4_last_error()) > 0);
                                        ++refused;
                                        continue;
                                    }
                                    ++accepted;
                                    if (method != CHAIN_FUSED || P.resident) continue;
                                    const int64_t V = prec == CHAIN_FP64 ? 2 : 4;
                                    const int64_t E =
                                        64 * int64_t(P.sites_per_lane) * P.waves_per_cluster;
                                    CHECK(P.tile >= 1 && P.tile + 2 * P.halo == E);
                                    CHECK(P.halo % V == 0 && P.tile % V == 0);
                                    CHECK(P.waves == (n + P.tile - 1) / P.tile);
                                    CHECK(P.kdepth >= 1 && P.kdepth <= 32);
                                }
    CHECK(accepted > 10000 && refused > 10000);

    // tableaus: reach is defined for valid ones, plans keep the reach
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 400; ++trial) {
        const int stages = 1 + trial % 8;
        chain_rk4_tableau t = random_tableau(rng, stages);
        for (int model : {int(CHAIN_QUARTIC), int(CHAIN_HARMONIC), int(CHAIN_QUARTIC_NNN), int(CHAIN_HARMONIC_NNN)}) {
            const int64_t reach = chain_rk4_tableau_reach(model, &t);
            CHECK(reach >= 0 && reach <= 2 * 2 * stages);
            for (int s : {0, 4, 8})
                for (int w : {0, 1, 4})
                    for (int k : {0, 1, 5, 21, 32}) {
                        chain_rk4_desc d = desc(1 << 20, model, trial % 2, s, w, k, 0,
                                                CHAIN_SCHEME_TABLEAU);
                        chain_rk4_plan P{};
                        if (chain_rk4_plan_for(&d, &t, &P) != CHAIN_OK) continue;
                        CHECK(P.halo >= (reach > 0 ? reach : 1) * P.kdepth);
                        CHECK(P.halo % (trial % 2 ? 4 : 2) == 0);
                    }
        }
        CHECK(chain_rk4_tableau_reach(CHAIN_ROESSLER, &t) == -1);
        t.a[stages > 1 ? 1 : 0][0] = NAN;
        t.b[0] = stages > 1 ? t.b[0] : NAN;
        CHECK(chain_rk4_tableau_reach(CHAIN_QUARTIC, &t) == -1);
    }
    chain_rk4_tableau bad{};
    bad.stages = 9;
    CHECK(chain_rk4_tableau_reach(CHAIN_QUARTIC, &bad) == -1);
    CHECK(chain_rk4_tableau_reach(CHAIN_QUARTIC, nullptr) == -1);

    // batch shapes
    for (int s : {-1, 0, 2, 4, 8, 16, 32})
        for (int k = -1; k <= 34; ++k)
            for (int flags : {0, 1, 2, 3, 4}) {
                chain_rk4_batch_desc bd{};
                bd.max_steps = 100;
                bd.sites_per_lane = s;
                bd.kdepth = k;
                bd.flags = flags;
                chain_rk4_batch_plan P{};
                if (chain_rk4_batch_plan_for(&bd, &P) != CHAIN_OK) continue;
                const int64_t E = 64 * int64_t(P.sites_per_lane) * P.waves_per_cluster;
                CHECK(P.halo % 4 == 0 && P.halo >= 2 * P.kdepth && E >= 4 * P.halo + 16);
                CHECK(chain_rk4_batch_clusters(1 << 20, s, k) >= 1);
                // the cut of assorted lengths: kept ranges tile [0, n)
                for (int64_t n : {int64_t(1), int64_t(3), int64_t(383), int64_t(1100),
                                  int64_t(4332), int64_t(65537), int64_t(1) << 33}) {
                    int64_t st[64], kp[64];
                    int32_t wv[64];
                    const int64_t G = chain_rk4_batch_layout(n, &bd, st, kp, wv, 64);
                    CHECK(G >= 1);
                    int64_t at = 0;
                    for (int64_t i = 0; i < G && i < 64; ++i) {
                        CHECK(st[i] == at && kp[i] > 0 && (wv[i] == 1 || wv[i] == P.waves_per_cluster));
                        at += kp[i];
                    }
                    if (G <= 64) CHECK(at == n);
                }
            }

    // validation of every call that takes a handle, a batch or pointers
    chain_rk4_desc d = desc(1000, 0, 0, 0, 0, 0, 0, 0);
    const size_t ws = chain_rk4_workspace_bytes(&d);
    CHECK(ws > 0);
    void *fake = reinterpret_cast<void *>(uintptr_t(1) << 20);
    chain_rk4 *h = nullptr;
    CHECK(chain_rk4_create(&d, nullptr, fake, fake, ws, nullptr, &h) == CHAIN_EINVAL);
    CHECK(chain_rk4_create(&d, fake, fake, fake, ws - 1, nullptr, &h) == CHAIN_ENOMEM);
    CHECK(chain_rk4_create(&d, static_cast<char *>(fake) + 8, fake, fake, ws, nullptr, &h) ==
          CHAIN_EINVAL);
    CHECK(chain_rk4_create(&d, fake, fake, static_cast<char *>(fake) + 16, ws, nullptr, &h) ==
          CHAIN_EINVAL);
    CHECK(chain_rk4_create(&d, fake, fake, fake, ws, nullptr, nullptr) == CHAIN_EINVAL);
    CHECK(h == nullptr);
    CHECK(chain_rk4_create3(&d, fake, fake, fake, fake, ws, nullptr, &h) == CHAIN_EINVAL);
    chain_rk4_desc r = desc(1000, CHAIN_ROESSLER, 0, 0, 0, 0, 0, 0);
    CHECK(chain_rk4_create(&r, fake, fake, fake, chain_rk4_workspace_bytes(&r), nullptr, &h) ==
          CHAIN_EINVAL);
    double e = 0.0;
    chain_rk4_plan P{};
    void *cq = nullptr, *cp = nullptr;
    CHECK(chain_rk4_step(nullptr, 1) == CHAIN_EINVAL);
    CHECK(chain_rk4_energy(nullptr, &e) == CHAIN_EINVAL);
    CHECK(chain_rk4_get_plan(nullptr, &P) == CHAIN_EINVAL);
    CHECK(chain_rk4_get_carries(nullptr, &cq, &cp) == CHAIN_EINVAL);
    CHECK(chain_rk4_set_stream(nullptr, nullptr) == CHAIN_EINVAL);
    CHECK(chain_rk4_set_tableau(nullptr, &bad) == CHAIN_EINVAL);
    CHECK(chain_rk4_destroy(nullptr) == CHAIN_OK);
    CHECK(chain_rk4_plan_for(&d, nullptr, nullptr) == CHAIN_EINVAL);
    chain_rk4_batch_desc bd{};
    bd.max_steps = 10;
    chain_rk4 *none[1] = {nullptr};
    chain_rk4_batch *b = nullptr;
    int64_t id = 0;
    CHECK(chain_rk4_batch_workspace_bytes(none, 1, &bd) == 0);
    CHECK(chain_rk4_batch_create(none, 1, &bd, fake, 1 << 20, nullptr, &b) == CHAIN_EINVAL);
    CHECK(chain_rk4_batch_create(nullptr, 0, &bd, fake, 1 << 20, nullptr, &b) == CHAIN_EINVAL);
    CHECK(chain_rk4_batch_step(nullptr, nullptr) == CHAIN_EINVAL);
    CHECK(chain_rk4_batch_check(nullptr) == CHAIN_EINVAL);
    CHECK(chain_rk4_batch_check_launch(nullptr, 0) == CHAIN_EINVAL);
    CHECK(chain_rk4_batch_last_launch(nullptr, &id) == CHAIN_EINVAL);
    CHECK(chain_rk4_batch_energy(nullptr, &e) == CHAIN_EINVAL);
    CHECK(chain_rk4_batch_rebind(nullptr, none, 1) == CHAIN_EINVAL);
    CHECK(chain_rk4_batch_destroy(nullptr) == CHAIN_OK);
    for (int code = -7; code <= 1; ++code) CHECK(chain_rk4_strerror(code) != nullptr);
    if (failures) return 1;
    std::printf("host driver: %ld plans accepted, %ld refused, all invariants hold\n", accepted,
                refused);
    return 0;
}
