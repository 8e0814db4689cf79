/*
 * chain_oracle.c -- plain, slow, obviously correct CPU reference for classical
 * RK4 stepping of a periodic one-dimensional chain with nearest-neighbour
 * coupling (Mulansky, "Optimizing Large-Scale ODE Simulations", Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the benchmark's
 * CPU-baseline leg are the only code that may load this library. It shares no
 * code, header or constant with the GPU library.
 *
 * Arithmetic is FP64 with no fused multiply-add (build with
 * -ffp-contract=off). Every per-site loop may run under OpenMP; the sites of a
 * sweep are independent, so the thread count never changes a result. Sums
 * over sites (the energy) run in index order on one thread.
 *
 * Models (homogeneous nearest-neighbour ODE, Sec. 2.1 Eq. 2, written as
 * dq_i/dt = p_i, dp_i/dt = F_i):
 *   quartic:  F_i = -(q_i + q_i^3) + (q_{i+1} - q_i)^3 - (q_i - q_{i-1})^3
 *   harmonic: F_i = -q_i + (q_{i+1} - 2 q_i + q_{i-1})
 * Next-nearest-neighbour variants (the generalisation named in Sec. 5): every
 * site is also bonded to its second neighbours, with the same bond potential:
 *   quartic NNN:  F_i = -(q_i + q_i^3) + (q_{i+1} - q_i)^3 - (q_i - q_{i-1})^3
 *                                      + (q_{i+2} - q_i)^3 - (q_i - q_{i-2})^3
 *   harmonic NNN: F_i = -q_i + (q_{i+1} - 2 q_i + q_{i-1})
 *                            + (q_{i+2} - 2 q_i + q_{i-2})
 * Periodic boundary (Sec. 3.1): site indices are taken mod N for every
 * N >= 1 (site 0's left neighbour is site N-1, and so on).
 *
 * Roessler chain (Sec. 3.1 Eq. 6-7), three coordinates per site:
 *   dx_i/dt = -y_i - z_i + (x_{i-1} - 2 x_i + x_{i+1})
 *   dy_i/dt = x_i + a y_i
 *   dz_i/dt = b + z_i (x_i - c)
 * with the paper's a = 0.2, b = 1, c = 9 passed in by the caller.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORACLE_QUARTIC = 0, ORACLE_HARMONIC = 1, ORACLE_QUARTIC_NNN = 3, ORACLE_HARMONIC_NNN = 4 };

static int64_t left_of(int64_t i, int64_t n) { return i == 0 ? n - 1 : i - 1; }
static int64_t right_of(int64_t i, int64_t n) { return i == n - 1 ? 0 : i + 1; }
/* i + d mod n, for any offset d */
static int64_t wrap(int64_t i, int64_t d, int64_t n)
{
    int64_t j = (i + d) % n;
    return j < 0 ? j + n : j;
}
static int is_nnn(int model) { return model == ORACLE_QUARTIC_NNN || model == ORACLE_HARMONIC_NNN; }

/* The force on one site from its own coordinate and its two neighbours'. */
static double force_site(int model, double qm, double q, double qp)
{
    if (model == ORACLE_QUARTIC) {
        double dr = qp - q;
        double dl = q - qm;
        return -(q + q * q * q) + dr * dr * dr - dl * dl * dl;
    }
    return -q + (qp - 2.0 * q + qm);
}

/* The same with the two second-neighbour bonds added. */
static double force_site_nnn(int model, double qmm, double qm, double q, double qp, double qpp)
{
    if (model == ORACLE_QUARTIC_NNN) {
        double dr = qp - q, dl = q - qm;
        double dr2 = qpp - q, dl2 = q - qmm;
        return -(q + q * q * q) + dr * dr * dr - dl * dl * dl + dr2 * dr2 * dr2 - dl2 * dl2 * dl2;
    }
    return -q + (qp - 2.0 * q + qm) + (qpp - 2.0 * q + qmm);
}

/* Force on site i of the ring, any model. */
static double force_at(int model, int64_t n, const double *q, int64_t i)
{
    if (is_nnn(model))
        return force_site_nnn(model, q[wrap(i, -2, n)], q[left_of(i, n)], q[i], q[right_of(i, n)],
                              q[wrap(i, 2, n)]);
    return force_site(model, q[left_of(i, n)], q[i], q[right_of(i, n)]);
}

/* Energy density of one site: kinetic + on-site potential + the potential of
 * the bond to the right neighbour (and, for the NNN models, of the bond to
 * the second neighbour on the right). Its gradient gives the force above. */
static double energy_site(int model, double q, double p, double qp, double qpp)
{
    double d = qp - q, d2 = qpp - q;
    if (model == ORACLE_QUARTIC)
        return p * p / 2.0 + q * q / 2.0 + q * q * q * q / 4.0 + d * d * d * d / 4.0;
    if (model == ORACLE_HARMONIC)
        return p * p / 2.0 + q * q / 2.0 + d * d / 2.0;
    if (model == ORACLE_QUARTIC_NNN)
        return p * p / 2.0 + q * q / 2.0 + q * q * q * q / 4.0 + d * d * d * d / 4.0 +
               d2 * d2 * d2 * d2 / 4.0;
    return p * p / 2.0 + q * q / 2.0 + d * d / 2.0 + d2 * d2 / 2.0;
}

/* Eq. 3: one evaluation of the right-hand side over the whole chain. */
static void rhs(int model, int64_t n, const double *q, const double *p,
                double *kq, double *kp, int threads)
{
    int64_t i;
#pragma omp parallel for num_threads(threads) schedule(static)
    for (i = 0; i < n; ++i) {
        kq[i] = p[i];
        kp[i] = force_at(model, n, q, i);
    }
}

/* Eq. 4: intermediate state y + a * dt * k. */
static void intermediate(int64_t n, const double *q, const double *p,
                         double a_dt, const double *kq, const double *kp,
                         double *Q, double *P, int threads)
{
    int64_t i;
#pragma omp parallel for num_threads(threads) schedule(static)
    for (i = 0; i < n; ++i) {
        Q[i] = q[i] + a_dt * kq[i];
        P[i] = p[i] + a_dt * kp[i];
    }
}

/* Public: the force F(q) over the whole chain. */
void oracle_force(int model, int64_t n, const double *q, double *f)
{
    int64_t i;
    for (i = 0; i < n; ++i)
        f[i] = force_at(model, n, q, i);
}

/*
 * Public: advance (q, p) in place by `steps` classical RK4 steps of size dt
 * (Sec. 2.2 Eq. 3-5 with the classical tableau c = (0, 1/2, 1/2, 1),
 * a21 = a32 = 1/2, a43 = 1, b = (1/6, 1/3, 1/3, 1/6)). dt may be negative.
 * Returns 0, or -1 if the work arrays cannot be allocated.
 */
int oracle_rk4_run(int model, int64_t n, double dt, int64_t steps,
                   double *q, double *p, int threads)
{
    double *buf, *k1q, *k1p, *k2q, *k2p, *k3q, *k3p, *k4q, *k4p, *Q, *P;
    int64_t s, i;
    if (n < 1 || steps < 0)
        return -1;
    if (threads < 1)
        threads = 1;
    buf = (double *)malloc(sizeof(double) * (size_t)n * 10);
    if (!buf)
        return -1;
    k1q = buf;          k1p = buf + n;
    k2q = buf + 2 * n;  k2p = buf + 3 * n;
    k3q = buf + 4 * n;  k3p = buf + 5 * n;
    k4q = buf + 6 * n;  k4p = buf + 7 * n;
    Q = buf + 8 * n;    P = buf + 9 * n;

    for (s = 0; s < steps; ++s) {
        rhs(model, n, q, p, k1q, k1p, threads);
        intermediate(n, q, p, dt / 2.0, k1q, k1p, Q, P, threads);
        rhs(model, n, Q, P, k2q, k2p, threads);
        intermediate(n, q, p, dt / 2.0, k2q, k2p, Q, P, threads);
        rhs(model, n, Q, P, k3q, k3p, threads);
        intermediate(n, q, p, dt, k3q, k3p, Q, P, threads);
        rhs(model, n, Q, P, k4q, k4p, threads);
        /* Eq. 5 */
#pragma omp parallel for num_threads(threads) schedule(static)
        for (i = 0; i < n; ++i) {
            q[i] = q[i] + (dt / 6.0) * (k1q[i] + 2.0 * k2q[i] + 2.0 * k3q[i] + k4q[i]);
            p[i] = p[i] + (dt / 6.0) * (k1p[i] + 2.0 * k2p[i] + 2.0 * k3p[i] + k4p[i]);
        }
    }
    free(buf);
    return 0;
}

/*
 * Public: advance (q, p) in place by `steps` steps of any explicit Runge-Kutta
 * method (Sec. 2.2 Eq. 3-5 with a general tableau; Sec. 2 notes the technique
 * applies to every explicit scheme). The method has s stages, coefficients
 * a (s x s, row-major; only the strictly lower triangle is read) and weights
 * b (s entries). Stage j evaluates the field at r + dt * sum_{m<j} a[j][m] k_m;
 * the step ends with r + dt * sum_m b[m] k_m. The models are autonomous, so
 * the nodes c play no part. Returns 0, or -1 on bad arguments or no memory.
 */
int oracle_rk_tableau_run(int model, int64_t n, double dt, int64_t steps, double *q, double *p,
                          int s, const double *a, const double *b, int threads)
{
    double *buf, *kq, *kp, *Q, *P;
    int64_t t, i;
    int j, m;
    if (n < 1 || steps < 0 || s < 1 || s > 16)
        return -1;
    if (threads < 1)
        threads = 1;
    buf = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(2 * s + 2));
    if (!buf)
        return -1;
    kq = buf;                          /* kq[j * n + i]: q part of k_j */
    kp = buf + (size_t)n * (size_t)s;  /* kp[j * n + i]: p part of k_j */
    Q = buf + (size_t)n * (size_t)(2 * s);
    P = Q + n;
    for (t = 0; t < steps; ++t) {
        for (j = 0; j < s; ++j) {
#pragma omp parallel for num_threads(threads) schedule(static) private(m)
            for (i = 0; i < n; ++i) {
                double sq = 0.0, sp = 0.0;
                for (m = 0; m < j; ++m) {
                    sq += a[j * s + m] * kq[(size_t)m * n + i];
                    sp += a[j * s + m] * kp[(size_t)m * n + i];
                }
                Q[i] = q[i] + dt * sq;
                P[i] = p[i] + dt * sp;
            }
            rhs(model, n, Q, P, kq + (size_t)j * n, kp + (size_t)j * n, threads);
        }
#pragma omp parallel for num_threads(threads) schedule(static) private(m)
        for (i = 0; i < n; ++i) {
            double sq = 0.0, sp = 0.0;
            for (m = 0; m < s; ++m) {
                sq += b[m] * kq[(size_t)m * n + i];
                sp += b[m] * kp[(size_t)m * n + i];
            }
            q[i] = q[i] + dt * sq;
            p[i] = p[i] + dt * sp;
        }
    }
    free(buf);
    return 0;
}

/*
 * Public: total energy H = sum_i e_i, summed in index order with Neumaier's
 * compensated summation (Neumaier 1974).
 */
double oracle_energy(int model, int64_t n, const double *q, const double *p)
{
    double sum = 0.0, comp = 0.0;
    int64_t i;
    for (i = 0; i < n; ++i) {
        double e = energy_site(model, q[i], p[i], q[right_of(i, n)], q[wrap(i, 2, n)]);
        double t = sum + e;
        if ((sum >= 0 ? sum : -sum) >= (e >= 0 ? e : -e))
            comp += (sum - t) + e;
        else
            comp += (e - t) + sum;
        sum = t;
    }
    return sum + comp;
}

/* ---------------------------------------------------------------------- */
/* Roessler chain                                                          */
/* ---------------------------------------------------------------------- */

/* Eq. 3 for the Roessler chain: local term (Eq. 6) plus coupling (Eq. 7). */
static void roessler_rhs(int64_t n, const double *x, const double *y, const double *z,
                         double a, double b, double c, double *kx, double *ky, double *kz,
                         int threads)
{
    int64_t i;
#pragma omp parallel for num_threads(threads) schedule(static)
    for (i = 0; i < n; ++i) {
        double xm = x[left_of(i, n)], xp = x[right_of(i, n)];
        kx[i] = -y[i] - z[i] + (xm - 2.0 * x[i] + xp);
        ky[i] = x[i] + a * y[i];
        kz[i] = b + z[i] * (x[i] - c);
    }
}

/* Public: the Roessler right-hand side over the whole chain. */
void oracle_roessler_rhs(int64_t n, const double *x, const double *y, const double *z,
                         double a, double b, double c, double *kx, double *ky, double *kz)
{
    roessler_rhs(n, x, y, z, a, b, c, kx, ky, kz, 1);
}

/* Eq. 4 for three components. */
static void intermediate3(int64_t n, const double *x, const double *y, const double *z,
                          double a_dt, const double *kx, const double *ky, const double *kz,
                          double *X, double *Y, double *Z, int threads)
{
    int64_t i;
#pragma omp parallel for num_threads(threads) schedule(static)
    for (i = 0; i < n; ++i) {
        X[i] = x[i] + a_dt * kx[i];
        Y[i] = y[i] + a_dt * ky[i];
        Z[i] = z[i] + a_dt * kz[i];
    }
}

/* Public: advance (x, y, z) in place by `steps` classical RK4 steps. */
int oracle_roessler_run(int64_t n, double dt, int64_t steps, double *x, double *y, double *z,
                        double a, double b, double c, int threads)
{
    double *buf, *k[4][3], *X, *Y, *Z;
    int64_t s, i;
    int j, m;
    if (n < 1 || steps < 0)
        return -1;
    if (threads < 1)
        threads = 1;
    buf = (double *)malloc(sizeof(double) * (size_t)n * 15);
    if (!buf)
        return -1;
    for (j = 0; j < 4; ++j)
        for (m = 0; m < 3; ++m)
            k[j][m] = buf + (size_t)n * (size_t)(3 * j + m);
    X = buf + 12 * n;
    Y = buf + 13 * n;
    Z = buf + 14 * n;

    for (s = 0; s < steps; ++s) {
        roessler_rhs(n, x, y, z, a, b, c, k[0][0], k[0][1], k[0][2], threads);
        intermediate3(n, x, y, z, dt / 2.0, k[0][0], k[0][1], k[0][2], X, Y, Z, threads);
        roessler_rhs(n, X, Y, Z, a, b, c, k[1][0], k[1][1], k[1][2], threads);
        intermediate3(n, x, y, z, dt / 2.0, k[1][0], k[1][1], k[1][2], X, Y, Z, threads);
        roessler_rhs(n, X, Y, Z, a, b, c, k[2][0], k[2][1], k[2][2], threads);
        intermediate3(n, x, y, z, dt, k[2][0], k[2][1], k[2][2], X, Y, Z, threads);
        roessler_rhs(n, X, Y, Z, a, b, c, k[3][0], k[3][1], k[3][2], threads);
#pragma omp parallel for num_threads(threads) schedule(static)
        for (i = 0; i < n; ++i) {
            x[i] = x[i] + (dt / 6.0) * (k[0][0][i] + 2.0 * k[1][0][i] + 2.0 * k[2][0][i] + k[3][0][i]);
            y[i] = y[i] + (dt / 6.0) * (k[0][1][i] + 2.0 * k[1][1][i] + 2.0 * k[2][1][i] + k[3][1][i]);
            z[i] = z[i] + (dt / 6.0) * (k[0][2][i] + 2.0 * k[1][2][i] + 2.0 * k[2][2][i] + k[3][2][i]);
        }
    }
    free(buf);
    return 0;
}
