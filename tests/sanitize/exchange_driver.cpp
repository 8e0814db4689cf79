// The host bookkeeping of the register-resident Roessler form
// (CHAIN_FLAG_EXCHANGE), under AddressSanitizer and UBSan with no GPU: the
// launchers are recording stand-ins (launch_stubs.cpp built with
// RECORD_EXCHANGE). Every exchange launch must start from the value its
// pass counters hold after the previous launch (base + passes - 1), and only
// the first launch of a handle clears them. Built and run by
// tests/test_sanitizers.py; exits 0 when every check holds.
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "chain_rk4.h"

extern std::vector<int> recorded_bases, recorded_passes;
extern int recorded_fills;

// The device queries handle creation makes, answered as one gfx950 device
// (these definitions take the place of the runtime's in this executable).
hipError_t hipGetDevice(int *dev) {
    *dev = 0;
    return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t *prop, int) {
    std::memset(prop, 0, sizeof *prop);
    std::strcpy(prop->gcnArchName, "gfx950");
    return hipSuccess;
}

static int failures = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "FAIL line %d: %s\n", __LINE__, #cond);         \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

int main() {
    chain_rk4_desc d{};
    d.n = 1 << 20;
    d.model = CHAIN_ROESSLER;
    d.prec = CHAIN_FP64;
    d.dt = 0.01;
    d.method = CHAIN_FUSED;
    d.flags = CHAIN_FLAG_EXCHANGE;
    const size_t ws = chain_rk4_workspace_bytes(&d);
    CHECK(ws > 0);
    // device pointers are never dereferenced on the host: aligned stand-ins
    void *fake = reinterpret_cast<void *>(uintptr_t(1) << 30);
    chain_rk4 *h = nullptr;
    CHECK(chain_rk4_create3(&d, fake, fake, fake, fake, ws, nullptr, &h) == CHAIN_OK);
    if (!h) {
        std::fprintf(stderr, "create failed: %s\n", chain_rk4_last_error());
        return 1;
    }
    chain_rk4_plan P{};
    CHECK(chain_rk4_get_plan(h, &P) == CHAIN_OK && P.exchange == 1 && P.kdepth == 13);
    const int fills_at_create = recorded_fills;     // the timeout word
    // calls of two or more steps take the exchange path
    const int64_t calls[] = {50, 2, 40, 27, 13, 1000, 3};
    for (int64_t k : calls) CHECK(chain_rk4_step(h, k) == CHAIN_OK);
    CHECK(recorded_bases.size() == 7);
    CHECK(recorded_fills == fills_at_create + 1);   // the first exchange call only
    int64_t expect = 0;
    for (size_t i = 0; i < recorded_bases.size(); ++i) {
        CHECK(recorded_passes[i] >= 2 && recorded_passes[i] % 2 == 0);
        CHECK(recorded_bases[i] == expect);
        expect += recorded_passes[i] - 1;
    }
    // near the top of the 32-bit range the counters are cleared first
    const int64_t big = int64_t(13) << 30;          // 2^30 passes of 13 steps
    CHECK(chain_rk4_step(h, big) == CHAIN_OK);
    CHECK(recorded_fills == fills_at_create + 2 && recorded_bases.back() == 0);
    CHECK(recorded_passes.back() == (1 << 30));
    CHECK(chain_rk4_step(h, 50) == CHAIN_OK);       // base 2^30 - 1: clears again
    CHECK(recorded_fills == fills_at_create + 3 && recorded_bases.back() == 0);
    CHECK(chain_rk4_step(h, 50) == CHAIN_OK);       // and counts on from there
    CHECK(recorded_fills == fills_at_create + 3);
    CHECK(recorded_bases.back() == recorded_passes[recorded_passes.size() - 2] - 1);
    CHECK(chain_rk4_destroy(h) == CHAIN_OK);
    if (failures) return 1;
    std::printf("exchange bookkeeping holds over %zu launches\n", recorded_bases.size());
    return 0;
}
