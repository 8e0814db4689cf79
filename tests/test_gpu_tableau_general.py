"""Explicit methods of 5, 7 and 8 stages through the tableau kernel (the
register bounds for six and for eight stage forces), against the oracle's
general stepper, through the C ABI.

The tableaus are random explicit ones (strictly lower-triangular A, weights
summing to one, drawn from fixed seeds): parity with the oracle holds for any
coefficients, so no literature method is needed to exercise these paths. The
oracle's general stepper itself is pinned by the methods of known order in
the CPU tests. FP64 bar: max-abs state error <= 1e-10 after 100 steps, energy
within 1e-12 relative; every cluster shape, depth and the per-stage path give
the same bits.
"""
import numpy as np
import pytest

import oracle
import workloads
from paper_1412_0544_amd import Chain

pytestmark = pytest.mark.gpu
TOL = 1e-10
OMODEL = {"quartic": oracle.QUARTIC, "quartic_nnn": oracle.QUARTIC_NNN}


def random_tableau(stages, seed):
    rng = np.random.default_rng(seed)
    a = np.tril(rng.uniform(-0.6, 0.9, (stages, stages)), -1)
    b = rng.uniform(0.05, 1.0, stages)
    b /= b.sum()
    return a, b


def run(q0, p0, steps, a, b, **kw):
    ch = Chain(q0, p0, 0.01, tableau=(a.tolist(), b.tolist()), **kw)
    ch.step(steps)
    e = ch.energy()
    out = [t.cpu().numpy().copy() for t in ch.state()]
    cq, cp = ch.carry_tensors()
    if cq is not None:
        out += [cq.cpu().numpy().copy(), cp.cpu().numpy().copy()]
    ch.close()
    return out, e


@pytest.mark.parametrize("stages", [5, 7, 8])
@pytest.mark.parametrize("model", ["quartic", "quartic_nnn"])
@pytest.mark.parametrize("n", [3, 257, 5003])
def test_matches_oracle(stages, model, n):
    a, b = random_tableau(stages, 100 + stages)
    q0, p0 = workloads.chain_ics(n, 21)
    qo, po = oracle.rk_tableau(OMODEL[model], q0, p0, 0.01, 100, a, b, threads=8)
    eo = oracle.energy(OMODEL[model], qo, po)
    for w in (1, 4):
        (q, p), e = run(q0, p0, 100, a, b, model=model, sites_per_lane=4, waves_per_cluster=w)
        assert np.abs(q - qo).max() <= TOL and np.abs(p - po).max() <= TOL, (w,)
        assert abs(e - eo) <= 1e-12 * abs(eo)


@pytest.mark.parametrize("stages", [5, 7, 8])
@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_shapes_depths_and_per_stage_path_identical_bits(stages, prec):
    a, b = random_tableau(stages, 200 + stages)
    dtype = np.float64 if prec == "fp64" else np.float32
    q0, p0 = workloads.chain_ics(20011, 22, dtype=dtype)
    ref, _ = run(q0, p0, 29, a, b, prec=prec, method="naive")
    for w in (1, 4):
        for k in (1, 3, 8):
            got, _ = run(q0, p0, 29, a, b, prec=prec, sites_per_lane=4, waves_per_cluster=w,
                         kdepth=k)
            for x, y in zip(got, ref):
                assert np.array_equal(x, y), (w, k)
