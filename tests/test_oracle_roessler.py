"""Pins of the oracle's Roessler chain (Sec. 3.1 Eq. 6-7, a = 0.2, b = 1,
c = 9) to facts outside the oracle: an independent high-order integrator,
the exact fixed point, the synchronized manifold, hand-expanded right-hand
sides, fourth-order convergence and translation symmetry."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import workloads

A, B, C = oracle.ROESSLER_ABC


def single_roessler(_t, v):
    x, y, z = v
    return [-y - z, x + A * y, B + z * (x - C)]


def chain_rhs_numpy(v, n):
    x, y, z = v[:n], v[n:2 * n], v[2 * n:]
    lap = np.roll(x, 1) + np.roll(x, -1) - 2 * x
    return np.concatenate([-y - z + lap, x + A * y, B + z * (x - C)])


def ics(n, seed):
    q, p = workloads.chain_ics(n, seed)
    r, _ = workloads.chain_ics(n, seed + 1000)
    return 5 * q, 5 * p, 0.5 + 0.5 * r


def test_synchronized_state_follows_the_single_oscillator():
    n, dt, steps = 8, 0.01, 500
    x0, y0, z0 = 1.0, -2.0, 0.3
    x, y, z = oracle.roessler_rk4(np.full(n, x0), np.full(n, y0), np.full(n, z0), dt, steps)
    # the coupling term vanishes exactly: every site stays identical
    assert np.array_equal(x, np.full(n, x[0])) and np.array_equal(z, np.full(n, z[0]))
    sol = solve_ivp(single_roessler, (0, dt * steps), [x0, y0, z0], method="DOP853",
                    rtol=1e-13, atol=1e-13)
    err = max(abs(x[0] - sol.y[0, -1]), abs(y[0] - sol.y[1, -1]), abs(z[0] - sol.y[2, -1]))
    assert err < 1e-6


def test_fixed_point_is_stationary():
    # equilibrium: x = -a y, z = -y, a y^2 + c y + b = 0
    yf = (-C + math.sqrt(C * C - 4 * A * B)) / (2 * A)
    n = 12
    x, y, z = oracle.roessler_rk4(np.full(n, -A * yf), np.full(n, yf), np.full(n, -yf), 0.01, 200)
    assert np.abs(x + A * yf).max() < 1e-12
    assert np.abs(y - yf).max() < 1e-12 and np.abs(z + yf).max() < 1e-12


def test_hand_expanded_rhs_on_tiny_rings():
    # N = 1: the coupling vanishes
    kx, ky, kz = oracle.roessler_rhs([0.4], [-1.1], [0.7])
    assert abs(kx[0] - (1.1 - 0.7)) < 1e-15
    assert abs(ky[0] - (0.4 + A * -1.1)) < 1e-15
    assert abs(kz[0] - (B + 0.7 * (0.4 - C))) < 1e-15
    # N = 2: both neighbours are the other site
    kx, _, _ = oracle.roessler_rhs([0.4, -0.3], [0.2, 0.1], [0.5, 0.6])
    assert abs(kx[0] - (-0.2 - 0.5 + 2 * (-0.3 - 0.4))) < 1e-15
    # N = 3: a genuine three-point stencil
    x = np.array([0.1, 0.9, -0.4])
    kx, _, _ = oracle.roessler_rhs(x, np.zeros(3), np.zeros(3))
    assert abs(kx[1] - (0.1 - 2 * 0.9 - 0.4)) < 1e-15
    assert abs(kx[0] - (-0.4 - 2 * 0.1 + 0.9)) < 1e-15


def test_rk4_matches_high_order_reference_integrator():
    n = 5
    x0, y0, z0 = ics(n, 3)
    sol = solve_ivp(lambda t, v: chain_rhs_numpy(v, n), (0, 1.0), np.concatenate([x0, y0, z0]),
                    method="DOP853", rtol=1e-13, atol=1e-13)
    x, y, z = oracle.roessler_rk4(x0, y0, z0, 0.005, 200)
    err = np.abs(np.concatenate([x, y, z]) - sol.y[:, -1]).max()
    assert err < 1e-7, err


def test_convergence_order_four():
    n = 16
    x0, y0, z0 = ics(n, 5)
    ref = np.concatenate(oracle.roessler_rk4(x0, y0, z0, 0.02 / 64, 64 * 25))
    errs = []
    for dt in (0.02, 0.01, 0.005):
        got = np.concatenate(oracle.roessler_rk4(x0, y0, z0, dt, int(round(0.5 / dt))))
        errs.append(np.abs(got - ref).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 3.7) & (orders < 4.3)), orders


def test_cyclic_shift_bitwise():
    n = 23
    x0, y0, z0 = ics(n, 8)
    base = oracle.roessler_rk4(x0, y0, z0, 0.01, 30)
    for s in (1, 7):
        sh = oracle.roessler_rk4(np.roll(x0, s), np.roll(y0, s), np.roll(z0, s), 0.01, 30)
        for a, b in zip(sh, base):
            assert np.array_equal(a, np.roll(b, s))


def test_light_cone_sites_equal_full_ring():
    n = 200
    x0, y0, z0 = ics(n, 9)
    full = oracle.roessler_rk4(x0, y0, z0, 0.01, 12)
    sites = [0, 99, 199]
    got = oracle.roessler_rk4_sites(x0, y0, z0, 0.01, 12, sites)
    for a, b in zip(got, full):
        assert np.array_equal(a, b[sites])


def test_exact_dependence_range_is_one_site_per_stage():
    """x couples to its neighbours directly in dx/dt, so the error front of a
    cut-off chain moves one site per stage (Sec. 2.3): four per step."""
    n, i, dt = 120, 60, 0.5
    x0, y0, z0 = ics(n, 6)
    for steps in (1, 2):
        base = oracle.roessler_rk4(x0, y0, z0, dt, steps)
        edge = 4 * steps
        for d in (edge, -edge, edge + 1, -(edge + 1)):
            v = [x0.copy(), y0.copy(), z0.copy()]
            v[0][i + d] += 0.1
            a = oracle.roessler_rk4(*v, dt, steps)
            moved = any(a[k][i] != base[k][i] for k in range(3))
            assert moved == (abs(d) <= edge), (steps, d)
