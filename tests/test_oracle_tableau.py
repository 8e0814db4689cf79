"""Pins of the oracle's general explicit Runge-Kutta stepper (any Butcher
tableau; Sec. 2 notes the cluster technique applies to every explicit
scheme) to facts outside the oracle: the literature tableaus satisfy their
order conditions, the classical tableau reproduces the dedicated RK4 path,
one step on a harmonic normal mode is the method's stability polynomial, the
observed convergence order is the tableau's, and the reach of one step
follows from the tableau's sparsity."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
import workloads


def tab(rows, b):
    s = len(b)
    a = np.zeros((s, s))
    for j, row in enumerate(rows):
        for m, v in enumerate(row):
            a[j + 1, m] = float(Fr(v))
    return a, np.array([float(Fr(x)) for x in b])


# Literature tableaus (strictly lower triangle row by row, then the weights).
TABLEAUS = {
    "midpoint": (tab([["1/2"]], ["0", "1"]), 2),
    "heun2": (tab([["1"]], ["1/2", "1/2"]), 2),
    "kutta3": (tab([["1/2"], ["-1", "2"]], ["1/6", "2/3", "1/6"]), 3),
    "ssprk3": (tab([["1"], ["1/4", "1/4"]], ["1/6", "1/6", "2/3"]), 3),
    "rk4": (tab([["1/2"], ["0", "1/2"], ["0", "0", "1"]], ["1/6", "1/3", "1/3", "1/6"]), 4),
    "rk4_38": (tab([["1/3"], ["-1/3", "1"], ["1", "-1", "1"]], ["1/8", "3/8", "3/8", "1/8"]), 4),
    # Dormand-Prince 5(4), the fifth-order solution (its seventh stage has
    # weight zero and is left out)
    "dopri5": (tab([["1/5"],
                    ["3/40", "9/40"],
                    ["44/45", "-56/15", "32/9"],
                    ["19372/6561", "-25360/2187", "64448/6561", "-212/729"],
                    ["9017/3168", "-355/33", "46732/5247", "49/176", "-5103/18656"]],
                   ["35/384", "0", "500/1113", "125/192", "-2187/6784", "11/84"]), 5),
}


@pytest.mark.parametrize("name", sorted(TABLEAUS))
def test_literature_tableaus_satisfy_their_order_conditions(name):
    (a, b), order = TABLEAUS[name]
    c = a.sum(axis=1)
    conds = [b.sum() - 1]
    if order >= 2:
        conds.append(b @ c - 1 / 2)
    if order >= 3:
        conds += [b @ c ** 2 - 1 / 3, b @ a @ c - 1 / 6]
    if order >= 4:
        conds += [b @ c ** 3 - 1 / 4, b @ (c * (a @ c)) - 1 / 8, b @ a @ c ** 2 - 1 / 12,
                  b @ a @ a @ c - 1 / 24]
    if order >= 5:
        conds += [b @ c ** 4 - 1 / 5, b @ (c ** 2 * (a @ c)) - 1 / 10,
                  b @ ((a @ c) ** 2) - 1 / 20, b @ (c * (a @ c ** 2)) - 1 / 15,
                  b @ a @ c ** 3 - 1 / 20, b @ (c * (a @ a @ c)) - 1 / 30,
                  b @ a @ (c * (a @ c)) - 1 / 40, b @ a @ a @ c ** 2 - 1 / 60,
                  b @ a @ a @ a @ c - 1 / 120]
    assert np.abs(conds).max() < 1e-14, conds


def test_classical_tableau_reproduces_the_rk4_path():
    (a, b), _ = TABLEAUS["rk4"]
    q0, p0 = workloads.chain_ics(300, 1)
    for model in (oracle.QUARTIC, oracle.QUARTIC_NNN):
        q1, p1 = oracle.rk_tableau(model, q0, p0, 0.01, 100, a, b)
        q2, p2 = oracle.rk4(model, q0, p0, 0.01, 100)
        assert max(abs(q1 - q2).max(), abs(p1 - p2).max()) < 1e-13


def stability_matrix(a, b, z):
    """R(Z) = I + sum_m (b^T a^{m-1} 1) Z^m: one step of the method on the
    linear system r' = (Z/dt) r (a is nilpotent, so the sum ends at m = s)."""
    s = b.size
    out = np.eye(z.shape[0])
    zm = np.eye(z.shape[0])
    am = np.eye(s)
    for _ in range(s):
        zm = zm @ z
        out = out + (b @ am @ np.ones(s)) * zm
        am = am @ a
    return out


@pytest.mark.parametrize("name", sorted(TABLEAUS))
@pytest.mark.parametrize("model,m", [(oracle.HARMONIC, 3), (oracle.HARMONIC_NNN, 5)])
def test_normal_mode_follows_the_stability_polynomial(name, model, m):
    (a, b), _ = TABLEAUS[name]
    n, dt, steps = 32, 0.1, 60
    th = 2 * np.pi * m / n
    w2 = 1 + 4 * np.sin(th / 2) ** 2 + (4 * np.sin(th) ** 2 if model == oracle.HARMONIC_NNN else 0)
    i = np.arange(n)
    a0, b0 = 0.5, -0.3
    q, p = oracle.rk_tableau(model, a0 * np.cos(th * i), b0 * np.cos(th * i), dt, steps, a, b)
    R = stability_matrix(a, b, dt * np.array([[0.0, 1.0], [-w2, 0.0]]))
    ab = np.linalg.matrix_power(R, steps) @ np.array([a0, b0])
    np.testing.assert_allclose(q, ab[0] * np.cos(th * i), rtol=0, atol=1e-12)
    np.testing.assert_allclose(p, ab[1] * np.cos(th * i), rtol=0, atol=1e-12)


@pytest.mark.parametrize("name", sorted(TABLEAUS))
def test_convergence_order(name):
    (a, b), order = TABLEAUS[name]
    q0, p0 = workloads.chain_ics(16, 4)
    # the fifth-order method reaches its asymptotic rate at smaller steps
    dts = (0.025, 0.0125, 0.00625) if order == 5 else (0.1, 0.05, 0.025)
    ref = oracle.rk_tableau(oracle.QUARTIC, q0, p0, dts[-1] / 32, int(round(32 / dts[-1])),
                            *TABLEAUS["dopri5"][0])
    errs = []
    for dt in dts:
        q, p = oracle.rk_tableau(oracle.QUARTIC, q0, p0, dt, int(round(1.0 / dt)), a, b)
        errs.append(max(abs(q - ref[0]).max(), abs(p - ref[1]).max()))
    obs = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert abs(obs[-1] - order) < 0.35 and np.all(obs > order - 0.35), obs


def step_reach(a, b, rng):
    """Sites one step reaches to each side for dq/dt = p, dp/dt = F(q) with F
    reaching `rng` sites: the stage argument Q_j takes the reach of the
    momenta it combines, P_j that of the forces, each force adds rng."""
    s = b.size
    rq, rp = [0] * s, [0] * s
    for j in range(1, s):
        used = [m for m in range(j) if a[j, m] != 0]
        rq[j] = max([rp[m] for m in used], default=0)
        rp[j] = max([rq[m] + rng for m in used], default=0)
    used = [m for m in range(s) if b[m] != 0]
    return max(max(rp[m] for m in used), max(rq[m] + rng for m in used))


@pytest.mark.parametrize("name", sorted(TABLEAUS))
@pytest.mark.parametrize("model,rng", [(oracle.QUARTIC, 1), (oracle.QUARTIC_NNN, 2)])
def test_exact_reach_of_one_step(name, model, rng):
    (a, b), _ = TABLEAUS[name]
    reach = step_reach(a, b, rng)
    n, i, dt = 120, 60, 0.5
    q0, p0 = workloads.chain_ics(n, 8)
    base = oracle.rk_tableau(model, q0, p0, dt, 1, a, b)
    for d in (reach, -reach, reach + 1, -(reach + 1)):
        moved = False
        for which in (0, 1):
            qq, pp = q0.copy(), p0.copy()
            (qq, pp)[which][i + d] += 0.1
            r = oracle.rk_tableau(model, qq, pp, dt, 1, a, b)
            moved |= bool(r[0][i] != base[0][i] or r[1][i] != base[1][i])
        assert moved == (abs(d) <= reach), (d, reach)
