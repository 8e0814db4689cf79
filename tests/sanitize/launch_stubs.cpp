// Stand-ins for the kernel launchers of the HIP library, so that its host
// translation units (argument validation, workspace layout, planning, the
// batch tables) build and run on a CPU under the sanitizers. No path the
// host driver takes reaches a launch; each stub fails loudly if one does.
// Built with RECORD_EXCHANGE, the fill, the exchange launch and its capacity
// query instead record their calls (exchange_driver.cpp reads them), so the
// host bookkeeping of the exchange form runs without a GPU.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "launch.hpp"

#ifdef RECORD_EXCHANGE
std::vector<int> recorded_bases, recorded_passes;
int recorded_fills = 0;
#endif

namespace chainrk4 {

[[noreturn]] static void unreachable(const char *what) {
    std::fprintf(stderr, "stub launcher %s reached from a validation path\n", what);
    std::abort();
}

hipError_t launch_fused(int, int, int, int, const FusedPass &, hipStream_t) { unreachable("fused"); }
hipError_t launch_resident(int, int, const ResidentRun &, hipStream_t) { unreachable("resident"); }
hipError_t launch_naive_step(int, int, StateRef, const NaiveBufs &, int64_t, double, hipStream_t) {
    unreachable("naive");
}
hipError_t launch_tableau(int, int, int, int, const FusedPass &, const TabArgs &, hipStream_t) {
    unreachable("tableau");
}
hipError_t launch_naive_tableau_step(int, int, StateRef, const NaiveTabBufs &, int64_t, double,
                                     const TabArgs &, hipStream_t) {
    unreachable("naive tableau");
}
hipError_t launch_fused_roessler(int, int, const FusedPass &, hipStream_t) { unreachable("roessler"); }
hipError_t launch_naive_roessler_step(StateRef, const NaiveBufs &, int64_t, double, hipStream_t) {
    unreachable("naive roessler");
}
#ifdef RECORD_EXCHANGE
hipError_t launch_exchange_roessler(int, int, const ExchangeRun &a, hipStream_t) {
    recorded_bases.push_back(a.base);
    recorded_passes.push_back(a.passes);
    return hipSuccess;
}
int exchange_capacity_roessler(int, int) { return 1 << 20; }
#else
hipError_t launch_exchange_roessler(int, int, const ExchangeRun &, hipStream_t) {
    unreachable("exchange roessler");
}
int exchange_capacity_roessler(int, int) { unreachable("exchange capacity"); }
#endif
int energy_blocks(int64_t) { unreachable("energy_blocks"); }
hipError_t launch_energy(int, int, StateRef, int64_t, double *, double *, hipStream_t) {
    unreachable("energy");
}
#ifdef RECORD_EXCHANGE
hipError_t launch_fill_zero(void *, size_t, hipStream_t) {
    ++recorded_fills;
    return hipSuccess;
}
#else
hipError_t launch_fill_zero(void *, size_t, hipStream_t) { unreachable("fill_zero"); }
#endif
int persistent_capacity(int, int, int, bool) { unreachable("persistent_capacity"); }
hipError_t launch_persistent(int, int, int, int, const BatchArgs &, hipStream_t) {
    unreachable("persistent");
}

}  // namespace chainrk4
