"""Next-nearest-neighbour chains on the GPU against the oracle, through the
C ABI: every site also bonded to its second neighbours (the generalisation of
Sec. 5; the overlap per side doubles).

FP64 bar as for the nearest-neighbour chains: max-abs state error <= 1e-10
after 100 steps, energy within 1e-12 relative; every GPU path gives the same
bits. FP32 with compensated update: <= 1e-5 against the FP64 oracle.
"""
import functools

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1412_0544_amd import Batch, Chain, ChainError

pytestmark = pytest.mark.gpu
TOL = 1e-10
MODELS = {"quartic_nnn": oracle.QUARTIC_NNN, "harmonic_nnn": oracle.HARMONIC_NNN}


def gpu_run(q0, p0, dt, steps, **kw):
    ch = Chain(q0, p0, dt, **kw)
    ch.step(steps)
    e = ch.energy()
    q, p = (t.cpu().numpy() for t in ch.state())
    plan = ch.plan()
    cq, cp = ch.carry_tensors()
    carries = None if cq is None else (cq.cpu().numpy(), cp.cpu().numpy())
    ch.close()
    return q, p, e, plan, carries


@functools.lru_cache(maxsize=None)
def oracle_run(model, n, seed, dt, steps):
    q0, p0 = workloads.chain_ics(n, seed)
    return oracle.rk4(MODELS[model], q0, p0, dt, steps, threads=8)


def maxerr(a, b):
    return float(np.max(np.abs(a - b))) if a.size else 0.0


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 64, 257, 1000, 5003, 20011])
@pytest.mark.parametrize("sites,waves,depth", [(4, 1, 1), (8, 2, 3), (16, 1, 8), (8, 4, 16),
                                               (4, 8, 4), (16, 8, 12), (8, 4, 32), (2, 1, 4),
                                               (2, 4, 8)])
def test_quartic_nnn_fused_matches_oracle(n, sites, waves, depth):
    q0, p0 = workloads.chain_ics(n, 1)
    q, p, e, plan, _ = gpu_run(q0, p0, 0.01, 100, model="quartic_nnn", sites_per_lane=sites,
                               waves_per_cluster=waves, kdepth=depth)
    assert plan["resident"] == 0 and plan["halo"] == 4 * plan["kdepth"]  # a multiple of 2 sites
    qo, po = oracle_run("quartic_nnn", n, 1, 0.01, 100)
    assert maxerr(q, qo) <= TOL and maxerr(p, po) <= TOL
    eo = oracle.energy(oracle.QUARTIC_NNN, qo, po)
    assert abs(e - eo) <= 1e-12 * abs(eo)


@pytest.mark.parametrize("n", [1, 5, 640, 4099])
def test_harmonic_nnn_fused_matches_oracle(n):
    q0, p0 = workloads.chain_ics(n, 2)
    q, p, e, _, _ = gpu_run(q0, p0, 0.05, 100, model="harmonic_nnn", sites_per_lane=8, kdepth=4)
    qo, po = oracle_run("harmonic_nnn", n, 2, 0.05, 100)
    assert maxerr(q, qo) <= TOL and maxerr(p, po) <= TOL
    eo = oracle.energy(oracle.HARMONIC_NNN, qo, po)
    assert abs(e - eo) <= 1e-12 * abs(eo)


@pytest.mark.parametrize("model", ["quartic_nnn", "harmonic_nnn"])
@pytest.mark.parametrize("n", [1, 2, 3, 1000, 30011])
def test_every_path_identical_bits(model, n):
    q0, p0 = workloads.chain_ics(n, 3)
    ref = gpu_run(q0, p0, 0.01, 37, model=model)
    outs = [gpu_run(q0, p0, 0.01, 37, model=model, method="naive")]
    for s, w, k in [(4, 1, 2), (8, 1, 5), (16, 2, 3), (4, 8, 16), (8, 4, 24), (16, 4, 32),
                    (2, 1, 3), (2, 8, 16)]:
        outs.append(gpu_run(q0, p0, 0.01, 37, model=model, sites_per_lane=s,
                            waves_per_cluster=w, kdepth=k))
    for o in outs:
        assert np.array_equal(o[0], ref[0]) and np.array_equal(o[1], ref[1])
        assert o[2] == ref[2]


def test_split_calls_and_graph_replays():
    n = 9000
    q0, p0 = workloads.chain_ics(n, 4)
    one = gpu_run(q0, p0, 0.01, 60, model="quartic_nnn", kdepth=8)
    for graph in (False, True):
        ch = Chain(q0, p0, 0.01, model="quartic_nnn", kdepth=8, graph=graph)
        for k in (1, 7, 13, 39):
            ch.step(k)
        torch.cuda.synchronize()
        assert np.array_equal(ch.q.cpu().numpy(), one[0]), graph
        assert np.array_equal(ch.p.cpu().numpy(), one[1]), graph
        ch.close()


def test_time_reversal_and_shift_bitwise():
    n = 5000
    q0, p0 = workloads.chain_ics(n, 5)
    base = gpu_run(q0, p0, 0.01, 32, model="quartic_nnn", sites_per_lane=8, kdepth=4)
    back = gpu_run(q0, -p0, -0.01, 32, model="quartic_nnn", sites_per_lane=16, kdepth=8)
    assert np.array_equal(back[0], base[0]) and np.array_equal(back[1], -base[1])
    for s in (1, 2, 4999):
        sh = gpu_run(np.roll(q0, s), np.roll(p0, s), 0.01, 32, model="quartic_nnn",
                     sites_per_lane=8, kdepth=4)
        assert np.array_equal(sh[0], np.roll(base[0], s))


@pytest.mark.parametrize("n", [3, 1000, 20011])
def test_fp32_kahan_error_bound_and_identical_bits(n):
    q0, p0 = workloads.chain_ics(n, 6, dtype=np.float32)
    runs = [gpu_run(q0, p0, 0.01, 100, model="quartic_nnn", prec="fp32_kahan", **kw)
            for kw in (dict(), dict(sites_per_lane=4, waves_per_cluster=8, kdepth=12),
                       dict(method="naive"))]
    for r in runs[1:]:
        for a, b in zip(r[:2] + r[4], runs[0][:2] + runs[0][4]):
            assert np.array_equal(a, b)
    q = runs[0][0].astype(np.float64) - runs[0][4][0]
    p = runs[0][1].astype(np.float64) - runs[0][4][1]
    qo, po = oracle.rk4(oracle.QUARTIC_NNN, q0.astype(np.float64), p0.astype(np.float64),
                        0.01, 100)
    assert maxerr(q, qo) <= 1e-5 and maxerr(p, po) <= 1e-5


@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32"])
@pytest.mark.parametrize("n,shape", [(100003, (4, 1, 16)), (600011, (4, 4, 16)),
                                     (1 << 21, (8, 4, 16)), (5000, (2, 1, 14))])
def test_fp32_library_rows_identical_bits(prec, n, shape):
    """The library's shapes for FP32 chains with second-neighbour bonds (one
    wavefront up to 2^18 sites, four beyond) give the bits of the
    one-kernel-per-stage method, carries included."""
    q0, p0 = workloads.chain_ics(n, 8, dtype=np.float32)
    a = gpu_run(q0, p0, 0.01, 40, model="harmonic_nnn", prec=prec)
    pl = a[3]
    assert (pl["sites_per_lane"], pl["waves_per_cluster"], pl["kdepth"]) == shape
    b = gpu_run(q0, p0, 0.01, 40, model="harmonic_nnn", prec=prec, method="naive")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    if a[4] is not None:
        assert np.array_equal(a[4][0], b[4][0]) and np.array_equal(a[4][1], b[4][1])


def test_large_chain_sampled_sites():
    """N = 2^22, default plan, 100 steps: sampled sites vs the oracle's light
    cones (2 * 8 * 100 + 1 sites each)."""
    n = 1 << 22
    q0, p0 = workloads.chain_ics(n, 0)
    q, p, _, plan, _ = gpu_run(q0, p0, 0.01, 100, model="quartic_nnn")
    tile = plan["tile"]
    rng = np.random.default_rng(3)
    sites = np.unique(np.concatenate([[0, 1, n - 1, n - 2, tile - 1, tile, tile + 1],
                                      rng.integers(0, n, 16)]))
    qs, ps = oracle.rk4_sites(oracle.QUARTIC_NNN, q0, p0, 0.01, 100, sites)
    assert maxerr(q[sites], qs) <= TOL and maxerr(p[sites], ps) <= TOL


def test_batches_reject_nnn_chains():
    q0, p0 = workloads.chain_ics(2000, 0)
    ch = Chain(q0, p0, 0.01, model="quartic_nnn")
    with pytest.raises(ChainError):
        Batch([ch], max_steps=10)
    ch.close()
