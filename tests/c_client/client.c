/*
 * A plain C client of the library: no Python, no torch. It allocates the
 * chain state and the workspace with the HIP runtime, advances a quartic
 * chain (Sec. 2.1 Eq. 2, periodic, classical RK4) through the C ABI of
 * include/chain_rk4.h, and prints the energy and a few sites of the result.
 *
 * Usage: chain_client N STEPS DT
 * Initial state: q_i = 0.8 sin(0.37 i + 0.1), p_i = 0.5 cos(0.21 i).
 * Output: one line "energy0 E0", one line "energy E", then "site i q p" lines
 * for i = 0, 1, N/2, N-1 (printed with %.17g).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "chain_rk4.h"

#define HIP_OK(x)                                                        \
    do {                                                                 \
        hipError_t e_ = (x);                                             \
        if (e_ != hipSuccess) {                                          \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));      \
            return 2;                                                    \
        }                                                                \
    } while (0)

#define CHAIN_OK_OR_FAIL(x)                                              \
    do {                                                                 \
        int s_ = (x);                                                    \
        if (s_ != CHAIN_OK) {                                            \
            fprintf(stderr, "%s: %s (%s)\n", #x, chain_rk4_strerror(s_), \
                    chain_rk4_last_error());                             \
            return 3;                                                    \
        }                                                                \
    } while (0)

int main(int argc, char **argv)
{
    if (argc != 4) {
        fprintf(stderr, "usage: %s N STEPS DT\n", argv[0]);
        return 1;
    }
    const int64_t n = atoll(argv[1]);
    const int64_t steps = atoll(argv[2]);
    const double dt = atof(argv[3]);
    if (n < 1 || steps < 0) return 1;

    double *hq = (double *)malloc(sizeof(double) * (size_t)n);
    double *hp = (double *)malloc(sizeof(double) * (size_t)n);
    if (!hq || !hp) return 1;
    for (int64_t i = 0; i < n; ++i) {
        hq[i] = 0.8 * sin(0.37 * (double)i + 0.1);
        hp[i] = 0.5 * cos(0.21 * (double)i);
    }

    chain_rk4_desc d = {0};
    d.n = n;
    d.model = CHAIN_QUARTIC;
    d.prec = CHAIN_FP64;
    d.dt = dt;
    d.method = CHAIN_FUSED;
    const size_t ws_bytes = chain_rk4_workspace_bytes(&d);
    if (ws_bytes == 0) return 1;

    void *q = NULL, *p = NULL, *ws = NULL;
    HIP_OK(hipMalloc(&q, sizeof(double) * (size_t)n));
    HIP_OK(hipMalloc(&p, sizeof(double) * (size_t)n));
    HIP_OK(hipMalloc(&ws, ws_bytes));   /* hipMalloc returns 256-byte aligned memory */
    HIP_OK(hipMemcpy(q, hq, sizeof(double) * (size_t)n, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(p, hp, sizeof(double) * (size_t)n, hipMemcpyHostToDevice));

    chain_rk4 *h = NULL;
    CHAIN_OK_OR_FAIL(chain_rk4_create(&d, q, p, ws, ws_bytes, NULL, &h));
    double e0 = 0.0, e1 = 0.0;
    CHAIN_OK_OR_FAIL(chain_rk4_energy(h, &e0));
    CHAIN_OK_OR_FAIL(chain_rk4_step(h, steps));
    CHAIN_OK_OR_FAIL(chain_rk4_energy(h, &e1));   /* synchronises the stream */
    CHAIN_OK_OR_FAIL(chain_rk4_destroy(h));

    HIP_OK(hipMemcpy(hq, q, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hp, p, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost));
    printf("energy0 %.17g\n", e0);
    printf("energy %.17g\n", e1);
    const int64_t sites[4] = {0, 1, n / 2, n - 1};
    for (int k = 0; k < 4; ++k)
        printf("site %lld %.17g %.17g\n", (long long)sites[k], hq[sites[k]], hp[sites[k]]);

    HIP_OK(hipFree(q));
    HIP_OK(hipFree(p));
    HIP_OK(hipFree(ws));
    free(hq);
    free(hp);
    return 0;
}
