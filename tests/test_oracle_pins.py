"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Each test ties the oracle to a closed form, an exact invariant, a special case
solved by an independent library routine, or a convergence property of the
classical RK4 scheme (Sec. 2.2 Eq. 3-5). Together they are chosen so that a
dropped term, a wrong sign or coefficient, a wrong neighbour index or a wrong
stage weight fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.special import ellipj

import oracle
import workloads

Q, H = oracle.QUARTIC, oracle.HARMONIC
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Inputs
# --------------------------------------------------------------------------

def test_splitmix64_reference_vectors():
    want = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    got = workloads.splitmix64(0, np.arange(4, dtype=np.uint64))
    assert [int(x) for x in got] == want


def test_ics_range_and_interleave():
    q, p = workloads.chain_ics(1000, 7)
    assert q.min() >= -1.0 and q.max() < 1.0 and p.min() >= -1.0 and p.max() < 1.0
    u = workloads.uniform01(7, np.array([10, 11], dtype=np.uint64))
    assert q[5] == 2 * u[0] - 1 and p[5] == 2 * u[1] - 1
    assert abs(q.mean()) < 0.1 and abs(np.var(q) - 1 / 3) < 0.05


# --------------------------------------------------------------------------
# Harmonic chain: the RK4 map of one normal mode is known exactly.
# --------------------------------------------------------------------------

def _rk4_mode_matrix(omega, dt):
    """One classical RK4 step of q'' = -omega^2 q is the degree-4 Taylor
    polynomial of exp(dt*A), A = [[0, 1], [-omega^2, 0]]. Since A^2 = -omega^2 I
    it collapses to c0*I + c1*A."""
    z2 = (omega * dt) ** 2
    c0 = 1.0 - z2 / 2.0 + z2 * z2 / 24.0
    c1 = dt * (1.0 - z2 / 6.0)
    return np.array([[c0, c1], [-omega * omega * c1, c0]])


@pytest.mark.parametrize("n,m", [(64, 0), (64, 1), (64, 5), (64, 31), (64, 32), (7, 3)])
@pytest.mark.parametrize("dt", [0.05, 0.3])
def test_harmonic_normal_mode_exact_discrete_map(n, m, dt):
    steps = 200
    theta = 2 * math.pi * m / n
    omega = math.sqrt(1.0 + 4.0 * math.sin(theta / 2) ** 2)
    i = np.arange(n)
    # a standing wave with both position and momentum components
    a0, b0 = 0.7, -0.4
    q0 = a0 * np.cos(theta * i + 0.3)
    p0 = b0 * np.cos(theta * i + 0.3)
    q, p = oracle.rk4(H, q0, p0, dt, steps)
    ab = np.linalg.matrix_power(_rk4_mode_matrix(omega, dt), steps) @ np.array([a0, b0])
    np.testing.assert_allclose(q, ab[0] * np.cos(theta * i + 0.3), rtol=0, atol=1e-12)
    np.testing.assert_allclose(p, ab[1] * np.cos(theta * i + 0.3), rtol=0, atol=1e-12)


def test_harmonic_superposition_two_modes():
    n, dt, steps = 48, 0.2, 150
    i = np.arange(n)
    q0 = np.zeros(n)
    p0 = np.zeros(n)
    parts = []
    for m, a, b, ph in [(3, 0.5, 0.1, 0.0), (11, -0.2, 0.6, 1.1)]:
        th = 2 * math.pi * m / n
        om = math.sqrt(1 + 4 * math.sin(th / 2) ** 2)
        q0 += a * np.cos(th * i + ph)
        p0 += b * np.cos(th * i + ph)
        parts.append((th, ph, np.linalg.matrix_power(_rk4_mode_matrix(om, dt), steps) @ [a, b]))
    q, p = oracle.rk4(H, q0, p0, dt, steps)
    qw = sum(ab[0] * np.cos(th * i + ph) for th, ph, ab in parts)
    pw = sum(ab[1] * np.cos(th * i + ph) for th, ph, ab in parts)
    np.testing.assert_allclose(q, qw, atol=1e-12)
    np.testing.assert_allclose(p, pw, atol=1e-12)


def test_harmonic_energy_factor_per_step():
    """For one mode, each RK4 step multiplies the energy by exactly
    c0^2 + omega^2 c1^2 = 1 - z^6/72 + z^8/576 with z = omega*dt."""
    n, m, dt, steps = 64, 5, 0.3, 100
    th = 2 * math.pi * m / n
    om = math.sqrt(1 + 4 * math.sin(th / 2) ** 2)
    z = om * dt
    q0, p0 = workloads.mode_ics(n, "cos", 0.9, m)
    e0 = oracle.energy(H, q0, p0)
    q, p = oracle.rk4(H, q0, p0, dt, steps)
    want = e0 * (1 - z ** 6 / 72 + z ** 8 / 576) ** steps
    assert abs(oracle.energy(H, q, p) - want) <= 1e-12 * abs(want)
    # and the modal energy closed form: (N/2) * (b^2 + omega^2 a^2) / 2
    assert abs(e0 - (n / 2) * (om * om * 0.81) / 2) < 1e-12


# --------------------------------------------------------------------------
# Quartic chain: two exact invariant manifolds with elliptic-function solutions.
# --------------------------------------------------------------------------

def _cn_solution(amp, kappa, t):
    """Q'' = -Q - kappa Q^3, Q(0) = amp, Q'(0) = 0 has
    Q = amp cn(Omega t | m), Omega^2 = 1 + kappa amp^2, m = kappa amp^2 / (2 Omega^2)."""
    om = math.sqrt(1 + kappa * amp * amp)
    m = kappa * amp * amp / (2 * om * om)
    sn, cn, dn, _ = ellipj(om * t, m)
    return amp * cn, -amp * om * sn * dn


@pytest.mark.parametrize("kind,kappa,n", [("uniform", 1.0, 16), ("uniform", 1.0, 1),
                                          ("pi", 17.0, 16), ("pi", 17.0, 2)])
def test_quartic_invariant_manifold_and_elliptic_solution(kind, kappa, n):
    amp, t_end = 0.8, 10.0
    q0, p0 = workloads.mode_ics(n, kind, amp)
    errs = []
    for dt in (0.02, 0.01):
        q, p = oracle.rk4(Q, q0, p0, dt, int(round(t_end / dt)))
        sign = np.where(np.arange(n) % 2 == 0, 1.0, -1.0) if kind == "pi" else np.ones(n)
        # the manifold is kept exactly: every site carries the same |q|, |p|
        assert np.array_equal(q * sign, np.full(n, q[0]))
        assert np.array_equal(p * sign, np.full(n, p[0]))
        qe, pe = _cn_solution(amp, kappa, t_end)
        errs.append(max(abs(q[0] - qe), abs(p[0] - pe)))
    assert errs[1] < (1e-8 if kind == "uniform" else 2e-6)
    ratio = errs[0] / errs[1]
    assert 12.0 < ratio < 24.0, ratio       # fourth order: about 2^4


def test_quartic_mode_energies_closed_form():
    n, a, b = 12, 0.7, -0.3
    q = np.full(n, a)
    p = np.full(n, b)
    assert abs(oracle.energy(Q, q, p) - n * (b * b / 2 + a * a / 2 + a ** 4 / 4)) < 1e-13
    s = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    want = n * (b * b / 2 + a * a / 2 + 17 * a ** 4 / 4)
    assert abs(oracle.energy(Q, a * s, b * s) - want) < 1e-12


# --------------------------------------------------------------------------
# Consistency of force and energy; the integrator against an independent one.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("model", [Q, H])
def test_force_is_minus_energy_gradient(model):
    q, p = workloads.chain_ics(9, 11)
    f = oracle.force(model, q)
    h = 1e-6
    for i in range(q.size):
        qp = q.copy(); qp[i] += h
        qm = q.copy(); qm[i] -= h
        g = (oracle.energy(model, qp, p) - oracle.energy(model, qm, p)) / (2 * h)
        assert abs(g + f[i]) < 1e-8, (i, g, f[i])


def test_tiny_rings_hand_expanded_forces():
    # N = 1: both neighbours are the site itself, the bonds vanish
    for x in (-0.9, 0.3, 1.7):
        assert abs(oracle.force(Q, [x])[0] + (x + x ** 3)) < 1e-15 * (1 + abs(x) ** 3)
        assert oracle.force(H, [x])[0] == -x
    # N = 2: both neighbours are the other site
    q0, q1 = 0.35, -0.8
    f = oracle.force(Q, [q0, q1])
    assert abs(f[0] - (-(q0 + q0 ** 3) + 2 * (q1 - q0) ** 3)) < 1e-15
    assert abs(f[1] - (-(q1 + q1 ** 3) + 2 * (q0 - q1) ** 3)) < 1e-15
    fh = oracle.force(H, [q0, q1])
    assert abs(fh[0] - (-q0 + 2 * (q1 - q0))) < 1e-15
    # N = 3: every site couples to the two others
    a, b, c = 0.2, -0.5, 0.9
    f = oracle.force(Q, [a, b, c])
    assert abs(f[1] - (-(b + b ** 3) + (c - b) ** 3 - (b - a) ** 3)) < 1e-15
    assert abs(f[0] - (-(a + a ** 3) + (b - a) ** 3 - (a - c) ** 3)) < 1e-15


@pytest.mark.parametrize("model,n", [(Q, 5), (Q, 2), (H, 6)])
def test_rk4_matches_high_order_reference_integrator(model, n):
    q0, p0 = workloads.chain_ics(n, 1)

    def f(_t, y):
        return np.concatenate([y[n:], oracle.force(model, y[:n])])

    sol = solve_ivp(f, (0.0, 2.0), np.concatenate([q0, p0]), method="DOP853",
                    rtol=1e-13, atol=1e-13)
    q, p = oracle.rk4(model, q0, p0, 0.01, 200)
    err = max(abs(q - sol.y[:n, -1]).max(), abs(p - sol.y[n:, -1]).max())
    assert err < 1e-7
    # the oracle's energy is a constant of the exact flow of its force
    e = [oracle.energy(model, sol.y[:n, k], sol.y[n:, k]) for k in range(sol.y.shape[1])]
    assert max(e) - min(e) < 1e-11


def _order_run(model, dt_list, t_end=1.0):
    q0, p0 = workloads.chain_ics(32, 3)
    ref = oracle.rk4(model, q0, p0, dt_list[0] / 64, int(round(t_end * 64 / dt_list[0])))
    e0 = oracle.energy(model, q0, p0)
    serr, eerr = [], []
    for dt in dt_list:
        q, p = oracle.rk4(model, q0, p0, dt, int(round(t_end / dt)))
        serr.append(max(abs(q - ref[0]).max(), abs(p - ref[1]).max()))
        eerr.append(abs(oracle.energy(model, q, p) - e0))
    return np.array(serr), np.array(eerr)


def test_convergence_order_four():
    serr, eerr = _order_run(Q, [0.05, 0.025, 0.0125])
    orders = np.log2(serr[:-1] / serr[1:])
    assert np.all((orders > 3.8) & (orders < 4.3)), orders
    eorders = np.log2(eerr[:-1] / eerr[1:])
    assert np.all(eorders > 3.7), eorders


# --------------------------------------------------------------------------
# Symmetries.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("model", [Q, H])
def test_time_reversal_bitwise(model):
    q0, p0 = workloads.chain_ics(29, 5)
    qa, pa = oracle.rk4(model, q0, -p0, 0.01, 50)
    qb, pb = oracle.rk4(model, q0, p0, -0.01, 50)
    assert np.array_equal(qa, qb) and np.array_equal(pa, -pb)


def test_forward_then_backward_returns_with_fourth_order_error():
    q0, p0 = workloads.chain_ics(40, 2)
    errs = []
    for dt, n in ((0.02, 50), (0.01, 100)):
        q, p = oracle.rk4(Q, q0, p0, dt, n)
        q, p = oracle.rk4(Q, q, p, -dt, n)
        errs.append(max(abs(q - q0).max(), abs(p - p0).max()))
    assert errs[1] < 1e-7
    assert 10.0 < errs[0] / errs[1] < 40.0


@pytest.mark.parametrize("model", [Q, H])
def test_cyclic_shift_bitwise(model):
    q0, p0 = workloads.chain_ics(37, 9)
    q, p = oracle.rk4(model, q0, p0, 0.01, 40)
    for s in (1, 5, 36):
        qs, ps = oracle.rk4(model, np.roll(q0, s), np.roll(p0, s), 0.01, 40)
        assert np.array_equal(qs, np.roll(q, s)) and np.array_equal(ps, np.roll(p, s))


@pytest.mark.parametrize("model", [Q, H])
def test_reflection(model):
    q0, p0 = workloads.chain_ics(31, 4)
    q, p = oracle.rk4(model, q0, p0, 0.01, 100)
    qr, pr = oracle.rk4(model, q0[::-1], p0[::-1], 0.01, 100)
    np.testing.assert_allclose(qr[::-1], q, atol=1e-13)
    np.testing.assert_allclose(pr[::-1], p, atol=1e-13)


# --------------------------------------------------------------------------
# Host-side helpers of the oracle.
# --------------------------------------------------------------------------

def test_light_cone_sites_equal_full_ring():
    q0, p0 = workloads.chain_ics(300, 8)
    qf, pf = oracle.rk4(Q, q0, p0, 0.01, 20)
    sites = [0, 1, 150, 298, 299]
    qs, ps = oracle.rk4_sites(Q, q0, p0, 0.01, 20, sites)
    assert np.array_equal(qs, qf[sites]) and np.array_equal(ps, pf[sites])


def test_thread_count_does_not_change_bits():
    q0, p0 = workloads.chain_ics(5000, 6)
    a = oracle.rk4(Q, q0, p0, 0.01, 10, threads=1)
    b = oracle.rk4(Q, q0, p0, 0.01, 10, threads=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_zero_steps_is_identity_and_bad_args_raise():
    q0, p0 = workloads.chain_ics(10, 1)
    q, p = oracle.rk4(Q, q0, p0, 0.01, 0)
    assert np.array_equal(q, q0) and np.array_equal(p, p0)
    with pytest.raises(MemoryError):
        oracle.rk4(Q, q0, p0, 0.01, -1)


def test_roessler_ics_range_and_interleave():
    x, y, z = workloads.roessler_ics(3000, 9)
    for v in (x, y, z):
        assert v.min() >= -1.0 and v.max() < 1.0 and abs(v.mean()) < 0.1
    u = workloads.uniform01(9, np.array([15, 16, 17], dtype=np.uint64))
    assert (x[5], y[5], z[5]) == tuple(2 * u - 1)


def test_device_ic_generator_matches_host_on_cpu():
    """The torch version of the initial-state generator (used to make long
    chains on the device) gives the host generator's bits, across its chunk
    boundaries and in FP32."""
    import torch
    for n, chunk in ((1000, 64), (4097, 1 << 26), (1, 1)):
        q, p = workloads.chain_ics_torch(n, 11, "cpu", chunk=chunk)
        q0, p0 = workloads.chain_ics(n, 11)
        assert np.array_equal(q.numpy(), q0) and np.array_equal(p.numpy(), p0)
    q, _ = workloads.chain_ics_torch(300, 2, "cpu", torch.float32, chunk=7)
    assert np.array_equal(q.numpy(), workloads.chain_ics(300, 2, dtype=np.float32)[0])
