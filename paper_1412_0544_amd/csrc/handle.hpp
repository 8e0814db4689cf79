// handle.hpp -- host-side internals shared by the C-ABI translation units:
// the chain handle, its pass plan and the error helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>

#include "chain_rk4.h"
#include "launch.hpp"

namespace chainrk4 {

// Record a message for chain_rk4_last_error() and return `status`.
int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char *what);
size_t elem_bytes(int prec);
bool has_carries(int prec);    // the FP32 precisions: per-site carries in the workspace
size_t carry_bytes(int prec);  // bytes of one carry
bool is_gfx950(int dev);

#define HIP_TRY(expr)                                                  \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return ::chainrk4::hip_fail(e_, #expr);  \
    } while (0)

struct Plan {
    bool resident = false;
    int sites = 0, depth = 0, waves_per_cluster = 0;
    int64_t tile = 0, halo = 0, waves = 0;
    // CHAIN_FLAG_EXCHANGE: `waves` clusters with balanced tiles (cluster g
    // keeps 4*uq sites, 4*(uq+1) if g < ur); zone: kept sites at a cluster's
    // left end that its left neighbour reads
    bool exchange = false;
    int64_t uq = 0, ur = 0, zone = 0;
};

}  // namespace chainrk4

struct chain_rk4 {
    chain_rk4_desc d;
    hipStream_t stream;
    chainrk4::StateRef front, back;
    chainrk4::NaiveBufs naive;
    double *partials, *result;
    chainrk4::Plan plan;
    hipStream_t capture = nullptr;
    std::map<int64_t, hipGraphExec_t> graphs;
    bool has_tableau = false;     // CHAIN_SCHEME_TABLEAU: set by chain_rk4_set_tableau
    chainrk4::TabArgs tableau{};
    chainrk4::NaiveTabBufs naive_tab{};
    int32_t *xflags = nullptr;    // CHAIN_FLAG_EXCHANGE: per-cluster pass counters
    int64_t xbase = -1;           // value of every counter after the last call, -1 if
                                  // unknown (cleared before the next call)
    int32_t *xerror = nullptr;    // CHAIN_FLAG_EXCHANGE: sticky timeout word
};
