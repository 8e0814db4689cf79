"""Pins of the oracle's next-nearest-neighbour chains (every site bonded to
its first and second neighbours with the same bond potential; the
generalisation of Sec. 5, whose overlap is twice as long) to facts outside
the oracle: the exact RK4 map of a normal mode, force = -grad H, hand-expanded
forces on tiny rings, an independent high-order integrator, fourth-order
convergence, exact symmetries, and the doubled light cone."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import workloads

QN, HN = oracle.QUARTIC_NNN, oracle.HARMONIC_NNN


def rk4_mode_matrix(omega, dt):
    """The classical RK4 step of q'' = -omega^2 q: the degree-4 Taylor
    polynomial of exp(dt*A) with A = [[0, 1], [-omega^2, 0]]."""
    z2 = (omega * dt) ** 2
    c0 = 1.0 - z2 / 2.0 + z2 * z2 / 24.0
    c1 = dt * (1.0 - z2 / 6.0)
    return np.array([[c0, c1], [-omega * omega * c1, c0]])


@pytest.mark.parametrize("n,m", [(64, 1), (64, 7), (64, 16), (64, 32), (9, 2), (5, 1)])
def test_harmonic_nnn_normal_mode_exact_map(n, m):
    # a wave of wavenumber theta: the first-neighbour bonds give
    # 4 sin^2(theta/2), the second-neighbour bonds 4 sin^2(theta)
    dt, steps = 0.1, 150
    theta = 2 * math.pi * m / n
    omega = math.sqrt(1 + 4 * math.sin(theta / 2) ** 2 + 4 * math.sin(theta) ** 2)
    i = np.arange(n)
    a0, b0 = -0.6, 0.45
    q, p = oracle.rk4(HN, a0 * np.cos(theta * i + 0.2), b0 * np.cos(theta * i + 0.2), dt, steps)
    ab = np.linalg.matrix_power(rk4_mode_matrix(omega, dt), steps) @ np.array([a0, b0])
    np.testing.assert_allclose(q, ab[0] * np.cos(theta * i + 0.2), rtol=0, atol=1e-12)
    np.testing.assert_allclose(p, ab[1] * np.cos(theta * i + 0.2), rtol=0, atol=1e-12)


@pytest.mark.parametrize("model", [QN, HN])
@pytest.mark.parametrize("n", [5, 9])
def test_force_is_minus_energy_gradient(model, n):
    q, p = workloads.chain_ics(n, 12)
    f = oracle.force(model, q)
    h = 1e-6
    for i in range(n):
        qp = q.copy(); qp[i] += h
        qm = q.copy(); qm[i] -= h
        g = (oracle.energy(model, qp, p) - oracle.energy(model, qm, p)) / (2 * h)
        assert abs(g + f[i]) < 1e-8, (i, g, f[i])


def test_tiny_rings_hand_expanded_forces():
    # N = 1 and N = 2: every second neighbour is the site itself, so the
    # second-neighbour bonds vanish and the forces equal the NN chain's
    for q in ([0.7], [0.35, -0.8]):
        assert np.array_equal(oracle.force(QN, q), oracle.force(oracle.QUARTIC, q))
        assert np.array_equal(oracle.force(HN, q), oracle.force(oracle.HARMONIC, q))
    # N = 3: the second neighbours are the first neighbours the other way round
    a, b, c = 0.2, -0.5, 0.9
    f = oracle.force(QN, [a, b, c])
    want = -(b + b ** 3) + (c - b) ** 3 - (b - a) ** 3 + (a - b) ** 3 - (b - c) ** 3
    assert abs(f[1] - want) < 1e-15
    # N = 5: all four neighbours distinct
    x = np.array([0.1, 0.9, -0.4, 0.3, 0.2])
    f = oracle.force(QN, x)
    want = (-(x[2] + x[2] ** 3) + (x[3] - x[2]) ** 3 - (x[2] - x[1]) ** 3
            + (x[4] - x[2]) ** 3 - (x[2] - x[0]) ** 3)
    assert abs(f[2] - want) < 1e-15
    want0 = (-(x[0] + x[0] ** 3) + (x[1] - x[0]) ** 3 - (x[0] - x[4]) ** 3
             + (x[2] - x[0]) ** 3 - (x[0] - x[3]) ** 3)
    assert abs(f[0] - want0) < 1e-15
    fh = oracle.force(HN, x)
    assert abs(fh[4] - (-x[4] + (x[0] - 2 * x[4] + x[3]) + (x[1] - 2 * x[4] + x[2]))) < 1e-15


@pytest.mark.parametrize("model,n", [(QN, 7), (HN, 6)])
def test_rk4_matches_high_order_reference_integrator(model, n):
    q0, p0 = workloads.chain_ics(n, 2)

    def f(_t, y):
        return np.concatenate([y[n:], oracle.force(model, y[:n])])

    sol = solve_ivp(f, (0.0, 2.0), np.concatenate([q0, p0]), method="DOP853",
                    rtol=1e-13, atol=1e-13)
    q, p = oracle.rk4(model, q0, p0, 0.005, 400)
    assert max(abs(q - sol.y[:n, -1]).max(), abs(p - sol.y[n:, -1]).max()) < 1e-8
    e = [oracle.energy(model, sol.y[:n, k], sol.y[n:, k]) for k in range(sol.y.shape[1])]
    assert max(e) - min(e) < 1e-11


def test_convergence_order_four():
    q0, p0 = workloads.chain_ics(24, 3)
    ref = oracle.rk4(QN, q0, p0, 0.05 / 64, 64 * 20)
    e0 = oracle.energy(QN, q0, p0)
    serr, eerr = [], []
    for dt in (0.05, 0.025, 0.0125):
        q, p = oracle.rk4(QN, q0, p0, dt, int(round(1.0 / dt)))
        serr.append(max(abs(q - ref[0]).max(), abs(p - ref[1]).max()))
        eerr.append(abs(oracle.energy(QN, q, p) - e0))
    orders = np.log2(np.array(serr[:-1]) / np.array(serr[1:]))
    assert np.all((orders > 3.8) & (orders < 4.3)), orders
    assert np.all(np.log2(np.array(eerr[:-1]) / np.array(eerr[1:])) > 3.7)


@pytest.mark.parametrize("model", [QN, HN])
def test_symmetries_bitwise(model):
    q0, p0 = workloads.chain_ics(33, 5)
    q, p = oracle.rk4(model, q0, p0, 0.01, 40)
    qa, pa = oracle.rk4(model, q0, -p0, -0.01, 40)          # time reversal
    assert np.array_equal(qa, q) and np.array_equal(pa, -p)
    for s in (1, 2, 32):                                    # cyclic shift
        qs, ps = oracle.rk4(model, np.roll(q0, s), np.roll(p0, s), 0.01, 40)
        assert np.array_equal(qs, np.roll(q, s)) and np.array_equal(ps, np.roll(p, s))
    qr, pr = oracle.rk4(model, q0[::-1], p0[::-1], 0.01, 40)  # reflection
    np.testing.assert_allclose(qr[::-1], q, atol=1e-13)


def test_light_cone_is_twice_as_wide():
    n, steps = 400, 12
    q0, p0 = workloads.chain_ics(n, 8)
    qf, pf = oracle.rk4(QN, q0, p0, 0.01, steps)
    sites = [0, 1, 200, 398, 399]
    qs, ps = oracle.rk4_sites(QN, q0, p0, 0.01, steps, sites)
    assert np.array_equal(qs, qf[sites]) and np.array_equal(ps, pf[sites])


@pytest.mark.parametrize("model,reach", [(oracle.QUARTIC, 1), (oracle.HARMONIC, 1), (QN, 2), (HN, 2)])
def test_exact_dependence_range_per_step(model, reach):
    """dq/dt = p is local and only dp/dt couples sites, so the stage
    arguments Q of stages 1 and 2 differ from q by local terms only: a step
    reaches 2 * reach sites to each side (not 4 * reach, one per stage, as for
    a field that couples every coordinate). Checked exactly with a large dt,
    which makes every dependence visible."""
    n, i, dt = 200, 100, 0.5
    q0, p0 = workloads.chain_ics(n, 8)
    for steps in (1, 3):
        base = oracle.rk4(model, q0, p0, dt, steps)
        edge = 2 * reach * steps
        for d in (edge, -edge, edge + 1, -(edge + 1)):
            for which in (0, 1):
                qq, pp = q0.copy(), p0.copy()
                (qq, pp)[which][i + d] += 0.1
                a = oracle.rk4(model, qq, pp, dt, steps)
                moved = a[0][i] != base[0][i] or a[1][i] != base[1][i]
                if abs(d) > edge:
                    assert not moved, (steps, d, which)
            qq = q0.copy()
            qq[i + d] += 0.1
            a = oracle.rk4(model, qq, p0, dt, steps)
            if abs(d) == edge:
                assert a[1][i] != base[1][i], (steps, d)
