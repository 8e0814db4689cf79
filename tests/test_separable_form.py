"""The GPU kernels take an RK4 step in a regrouped form: for dq/dt = p the q
slopes of the stages are the p stage values, so the q stage arguments and the
q update are formed from p and the forces alone (no p stage values):

    Q2 = q + (h/2) p,       Q3 = Q2 + (h/2)^2 F1,      Q4 = q + h p + h (h/2) F2,
    q' = q + h p + (h^2/6)(F1 + F2 + F3),
    p' = p + (h/6)(2 (F1 + F2 + F3) + F4 - F1).

This is exact algebra on the classical method (Sec. 2.2 Eq. 3-5 with the
classical tableau), so the regrouped step, written out here in numpy FP64 with
the oracle's own force, must agree with the oracle's stage-by-stage step to
rounding. A mistake in any coefficient of the regrouping (h/2 for h, a
missing F term, h^2/2 for h^2/6) would show as an O(h^2) or larger error.
"""
import numpy as np
import pytest

import oracle
import workloads


def separable_step(model, q, p, h, c2=1.0 / 6.0):
    """One step in the regrouped form; c2 is the coefficient of h^2 (F1+F2+F3)."""
    F = lambda x: oracle.force(model, x)
    F1 = F(q)
    Q2 = q + (h / 2) * p
    F2 = F(Q2)
    Q3 = Q2 + (h / 2) ** 2 * F1
    F3 = F(Q3)
    Q4 = q + h * p + h * (h / 2) * F2
    F4 = F(Q4)
    s = F1 + F2 + F3
    return q + h * p + (h * h * c2) * s, p + (h / 6) * (2 * s + F4 - F1)


@pytest.mark.parametrize("model", [oracle.QUARTIC, oracle.HARMONIC, oracle.QUARTIC_NNN,
                                   oracle.HARMONIC_NNN])
@pytest.mark.parametrize("h", [0.01, -0.05, 0.2])
def test_regrouped_step_is_classical_rk4(model, h):
    q0, p0 = workloads.chain_ics(257, 3)
    q, p = q0.copy(), p0.copy()
    for _ in range(20):
        q, p = separable_step(model, q, p, h)
    qo, po = oracle.rk4(model, q0, p0, h, 20)
    assert np.abs(q - qo).max() < 1e-12 and np.abs(p - po).max() < 1e-12


def test_a_wrong_coefficient_is_seen():
    """The same comparison notices a regrouping with h^2/2 for h^2/6."""
    q0, p0 = workloads.chain_ics(64, 4)
    h = 0.01
    qo, _ = oracle.rk4(oracle.QUARTIC, q0, p0, h, 1)
    right, _ = separable_step(oracle.QUARTIC, q0, p0, h)
    wrong, _ = separable_step(oracle.QUARTIC, q0, p0, h, c2=0.5)
    assert np.abs(right - qo).max() < 1e-15
    assert np.abs(wrong - qo).max() > 1e-6
