/*
 * Drives every entry point of the CPU oracle on small rings (N = 1, 2, 3, 7
 * and 64; every model; one and several threads; the classical and two other
 * explicit tableaus; the Roessler chain) under AddressSanitizer and
 * UndefinedBehaviorSanitizer, built with tests/test_sanitizers.py. Exits 0
 * when every call succeeds and returns finite values; a sanitizer finding
 * aborts the run.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_force(int model, int64_t n, const double *q, double *f);
int oracle_rk4_run(int model, int64_t n, double dt, int64_t steps, double *q, double *p,
                   int threads);
int oracle_rk_tableau_run(int model, int64_t n, double dt, int64_t steps, double *q, double *p,
                          int s, const double *a, const double *b, int threads);
double oracle_energy(int model, int64_t n, const double *q, const double *p);
void oracle_roessler_rhs(int64_t n, const double *x, const double *y, const double *z,
                         double a, double b, double c, double *kx, double *ky, double *kz);
int oracle_roessler_run(int64_t n, double dt, int64_t steps, double *x, double *y, double *z,
                        double a, double b, double c, int threads);

static int failures = 0;

static void check(int ok, const char *what, int64_t n, int model) {
    if (!ok) {
        fprintf(stderr, "FAIL %s n=%lld model=%d\n", what, (long long)n, model);
        ++failures;
    }
}

/* Exactly n values in their own allocation, so an access past either end is
 * a heap overflow the address sanitizer reports. */
static double *values(int64_t n, unsigned seed) {
    double *v = malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        seed = seed * 1103515245u + 12345u;
        v[i] = ((seed >> 8) & 0xffff) / 32768.0 - 1.0;
    }
    return v;
}

static int all_finite(const double *v, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

int main(void) {
    const int64_t lengths[] = {1, 2, 3, 7, 64};
    const int models[] = {0, 1, 3, 4};
    /* classical RK4, Heun's method and Kutta's third-order method */
    const double rk4_a[16] = {0, 0, 0, 0, 0.5, 0, 0, 0, 0, 0.5, 0, 0, 0, 0, 1, 0};
    const double rk4_b[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};
    const double heun_a[4] = {0, 0, 1, 0};
    const double heun_b[2] = {0.5, 0.5};
    const double k3_a[9] = {0, 0, 0, 0.5, 0, 0, -1, 2, 0};
    const double k3_b[3] = {1.0 / 6, 2.0 / 3, 1.0 / 6};
    for (size_t li = 0; li < sizeof lengths / sizeof lengths[0]; ++li) {
        const int64_t n = lengths[li];
        for (size_t mi = 0; mi < sizeof models / sizeof models[0]; ++mi) {
            const int model = models[mi];
            for (int threads = 1; threads <= 3; threads += 2) {
                double *q = values(n, 1u + (unsigned)li), *p = values(n, 7u + (unsigned)mi);
                double *f = values(n, 3u);
                oracle_force(model, n, q, f);
                check(all_finite(f, n), "force", n, model);
                check(isfinite(oracle_energy(model, n, q, p)), "energy", n, model);
                check(oracle_rk4_run(model, n, 0.01, 5, q, p, threads) == 0, "rk4", n, model);
                check(oracle_rk4_run(model, n, -0.01, 0, q, p, threads) == 0, "rk4 0 steps", n,
                      model);
                check(oracle_rk_tableau_run(model, n, 0.02, 3, q, p, 4, rk4_a, rk4_b, threads) == 0,
                      "tableau rk4", n, model);
                check(oracle_rk_tableau_run(model, n, 0.02, 3, q, p, 2, heun_a, heun_b, threads) ==
                          0,
                      "tableau heun", n, model);
                check(oracle_rk_tableau_run(model, n, 0.02, 3, q, p, 3, k3_a, k3_b, threads) == 0,
                      "tableau kutta3", n, model);
                check(all_finite(q, n) && all_finite(p, n), "state", n, model);
                free(q);
                free(p);
                free(f);
            }
        }
        double *x = values(n, 11u), *y = values(n, 12u), *z = values(n, 13u);
        double *kx = values(n, 1u), *ky = values(n, 2u), *kz = values(n, 3u);
        oracle_roessler_rhs(n, x, y, z, 0.2, 1.0, 9.0, kx, ky, kz);
        check(all_finite(kx, n) && all_finite(ky, n) && all_finite(kz, n), "roessler rhs", n, 2);
        check(oracle_roessler_run(n, 0.01, 5, x, y, z, 0.2, 1.0, 9.0, 1) == 0, "roessler", n, 2);
        check(oracle_roessler_run(n, 0.01, 5, x, y, z, 0.2, 1.0, 9.0, 3) == 0, "roessler mt", n,
              2);
        check(all_finite(x, n) && all_finite(y, n) && all_finite(z, n), "roessler state", n, 2);
        free(x);
        free(y);
        free(z);
        free(kx);
        free(ky);
        free(kz);
    }
    /* invalid arguments are refused, not run */
    double q1[1] = {0.5}, p1[1] = {0.0};
    check(oracle_rk4_run(0, 0, 0.01, 1, q1, p1, 1) != 0, "n = 0 refused", 0, 0);
    check(oracle_rk4_run(0, 1, 0.01, -1, q1, p1, 1) != 0, "negative steps refused", 1, 0);
    check(oracle_rk_tableau_run(0, 1, 0.01, 1, q1, p1, 0, rk4_a, rk4_b, 1) != 0,
          "zero stages refused", 1, 0);
    if (failures) return 1;
    printf("oracle driver: all calls clean\n");
    return 0;
}
