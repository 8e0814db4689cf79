"""The Roessler chain (Sec. 3.1 Eq. 6-7) on the GPU against the oracle,
through the C ABI.

FP64 bar: max-abs state error <= 1e-10 after 100 steps. The fused kernel at
every cluster shape and depth and the one-kernel-per-stage method give the
same bits. At the paper's size (N = 2^20) sampled sites are checked against
the oracle, each from its own light cone.
"""
import functools

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1412_0544_amd import ChainError, RoesslerChain

pytestmark = pytest.mark.gpu
TOL = 1e-10


def gpu_run(ics, dt, steps, **kw):
    ch = RoesslerChain(*ics, dt, **kw)
    ch.step(steps)
    out = tuple(t.cpu().numpy() for t in ch.state())
    plan = ch.plan()
    ch.close()
    return out, plan


@functools.lru_cache(maxsize=None)
def oracle_run(n, seed, dt, steps):
    return oracle.roessler_rk4(*workloads.roessler_ics(n, seed), dt, steps, threads=8)


def maxerr(a, b):
    return max(float(np.max(np.abs(u - v))) for u, v in zip(a, b))


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 257, 1000, 5003, 20011])
@pytest.mark.parametrize("sites,waves,depth", [(4, 1, 1), (8, 2, 3), (16, 1, 8), (4, 8, 16),
                                               (4, 4, 12), (8, 4, 16), (16, 8, 12), (6, 4, 13),
                                               (6, 1, 5)])
def test_fused_matches_oracle(n, sites, waves, depth):
    ics = workloads.roessler_ics(n, 1)
    got, plan = gpu_run(ics, 0.01, 100, sites_per_lane=sites, waves_per_cluster=waves,
                        kdepth=depth)
    assert plan["resident"] == 0 and plan["sites_per_lane"] == sites
    assert maxerr(got, oracle_run(n, 1, 0.01, 100)) <= TOL


@pytest.mark.parametrize("n", [1, 5, 1000, 20011])
def test_naive_matches_oracle_and_fused_bits(n):
    ics = workloads.roessler_ics(n, 2)
    naive, _ = gpu_run(ics, 0.01, 100, method="naive")
    fused, _ = gpu_run(ics, 0.01, 100)
    assert maxerr(naive, oracle_run(n, 2, 0.01, 100)) <= TOL
    for a, b in zip(naive, fused):
        assert np.array_equal(a, b)


def test_shapes_depths_and_step_splits_identical_bits():
    n = 3 * 2048 + 77
    ics = workloads.roessler_ics(n, 3)
    ref, _ = gpu_run(ics, 0.01, 37)
    for s, w, k in [(4, 1, 1), (4, 2, 5), (8, 8, 16), (16, 4, 7), (8, 1, 2), (6, 4, 21),
                    (6, 2, 9)]:
        got, _ = gpu_run(ics, 0.01, 37, sites_per_lane=s, waves_per_cluster=w, kdepth=k)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), (s, w, k)
    # 37 steps as 1 + 16 + 20 calls, and replayed from captured graphs
    for graph in (False, True):
        ch = RoesslerChain(*ics, 0.01, graph=graph)
        for k in (1, 16, 20):
            ch.step(k)
        torch.cuda.synchronize()
        for a, b in zip(ref, ch.state()):
            assert np.array_equal(a, b.cpu().numpy()), graph
        ch.close()


def test_synchronized_chain_and_fixed_point():
    """Identical sites stay identical (the coupling term vanishes exactly);
    the fixed point of the single oscillator stays put."""
    n = 5000
    ch = RoesslerChain(np.full(n, 1.0), np.full(n, -2.0), np.full(n, 0.3), 0.01)
    ch.step(500)
    x, y, z = (t.cpu().numpy() for t in ch.state())
    assert np.all(x == x[0]) and np.all(y == y[0]) and np.all(z == z[0])
    ch.close()
    xo, yo, zo = oracle.roessler_rk4(np.ones(3), np.full(3, -2.0), np.full(3, 0.3), 0.01, 500)
    assert abs(x[0] - xo[0]) < 1e-11 and abs(y[0] - yo[0]) < 1e-11 and abs(z[0] - zo[0]) < 1e-11
    a, b, c = oracle.ROESSLER_ABC
    yf = (-c + np.sqrt(c * c - 4 * a * b)) / (2 * a)
    ch = RoesslerChain(np.full(n, -a * yf), np.full(n, yf), np.full(n, -yf), 0.01)
    ch.step(200)
    x, y, z = (t.cpu().numpy() for t in ch.state())
    assert np.abs(x + a * yf).max() < 1e-12 and np.abs(y - yf).max() < 1e-12
    assert np.abs(z + yf).max() < 1e-12
    ch.close()


def test_translation_symmetry_bitwise():
    n = 10007
    x0, y0, z0 = workloads.roessler_ics(n, 4)
    a, _ = gpu_run((x0, y0, z0), 0.01, 64)
    b, _ = gpu_run(tuple(np.roll(v, 1234) for v in (x0, y0, z0)), 0.01, 64)
    for u, v in zip(a, b):
        assert np.array_equal(np.roll(u, 1234), v)


def test_paper_size_sampled_sites():
    """N = 2^20, dt = 0.01, T = 50 steps (the paper's protocol), default
    plan: sampled sites vs the oracle's light cones."""
    n = 1 << 20
    ics = workloads.roessler_ics(n, 0)
    got, plan = gpu_run(ics, 0.01, 50)
    tile = plan["tile"]
    rng = np.random.default_rng(1)
    sites = np.unique(np.concatenate([[0, 1, n - 1, tile - 1, tile, 2 * tile],
                                      rng.integers(0, n, 24)]))
    want = oracle.roessler_rk4_sites(*ics, 0.01, 50, sites)
    assert maxerr(tuple(g[sites] for g in got), want) <= TOL
    assert all(np.all(np.isfinite(g)) for g in got)


def test_long_chain_plan_sampled_sites():
    """N = 2^22 (past the paper's size): the long-chain plan, 8 sites per lane
    at depth 25, against the oracle's light cones at sampled sites."""
    n = 1 << 22
    ics = workloads.roessler_ics(n, 2)
    got, plan = gpu_run(ics, 0.01, 60)
    assert (plan["sites_per_lane"], plan["waves_per_cluster"], plan["kdepth"]) == (8, 4, 25)
    tile = plan["tile"]
    rng = np.random.default_rng(2)
    sites = np.unique(np.concatenate([[0, 1, n - 1, tile - 1, tile, 2 * tile],
                                      rng.integers(0, n, 24)]))
    want = oracle.roessler_rk4_sites(*ics, 0.01, 60, sites)
    assert maxerr(tuple(g[sites] for g in got), want) <= TOL
    assert all(np.all(np.isfinite(g)) for g in got)


def test_roessler_rejects_energy_and_batches():
    from paper_1412_0544_amd import Batch
    ch = RoesslerChain(*workloads.roessler_ics(100, 0), 0.01)
    import ctypes
    from paper_1412_0544_amd import _lib as L
    e = ctypes.c_double()
    assert L.lib().chain_rk4_energy(ch.handle, ctypes.byref(e)) == L.CHAIN_EINVAL
    with pytest.raises(ChainError):
        Batch([ch], max_steps=10)
    ch.close()


# The register-resident form (CHAIN_FLAG_EXCHANGE): every cluster stays in
# registers for a whole step call and swaps only edge sites between passes.
# The same per-site arithmetic as the fused passes: the same bits.
@pytest.mark.parametrize("n,sites,waves,depth,steps", [
    (2051, 4, 2, 1, 2), (4001, 4, 1, 6, 37), (9000, 4, 4, 13, 50), (20011, 4, 4, 25, 50),
    (30011, 8, 2, 20, 61), (40003, 4, 8, 32, 64), (8195, 4, 4, 16, 1000), (2000, 4, 4, 25, 50),
    (20011, 4, 4, 25, 1), (20011, 4, 4, 25, 3), (9000, 6, 4, 13, 50), (30011, 6, 4, 21, 61),
    (20011, 6, 2, 8, 37)])
def test_exchange_equals_fused_bits(n, sites, waves, depth, steps):
    ics = workloads.roessler_ics(n, 5)
    kw = dict(sites_per_lane=sites, waves_per_cluster=waves, kdepth=depth)
    ref, _ = gpu_run(ics, 0.01, steps, **kw)
    ch = RoesslerChain(*ics, 0.01, exchange=True, **kw)
    assert ch.plan()["exchange"] == 1
    ch.step(steps)
    ch.check()
    got = tuple(t.cpu().numpy() for t in ch.state())
    ch.close()
    for a, b in zip(got, ref):
        assert np.array_equal(a, b), (n, sites, waves, depth, steps)


def test_exchange_against_the_oracle_and_across_calls():
    n = 12011
    ics = workloads.roessler_ics(n, 6)
    ch = RoesslerChain(*ics, 0.01, exchange=True)
    for k in (30, 1, 69):                     # 100 steps in calls of 30, 1 and 69
        ch.step(k)
    ch.check()
    got = tuple(t.cpu().numpy() for t in ch.state())
    ch.close()
    assert maxerr(got, oracle_run(n, 6, 0.01, 100)) <= TOL
    g = RoesslerChain(*ics, 0.01, exchange=True, graph=True)
    for _ in range(3):                        # replayed graph, three times
        g.step(50)
    g.check()
    once = RoesslerChain(*ics, 0.01, exchange=True)
    once.step(150)
    once.check()
    for a, b in zip(g.state(), once.state()):
        assert torch.equal(a, b)


def test_exchange_counters_carry_over_many_calls():
    """The progress counters are not cleared between eager calls (each call
    starts from the value the last one left): 60 calls of 1 to 7 steps give
    the bits of one call over the same steps; on a graph handle, two graphs
    replayed in turn (each clears the counters) give them too."""
    n = 20011
    ics = workloads.roessler_ics(n, 7)
    ks = [1 + (5 * i) % 7 for i in range(60)]
    many = RoesslerChain(*ics, 0.01, exchange=True)
    for k in ks:
        many.step(k)
    many.check()
    once = RoesslerChain(*ics, 0.01, exchange=True)
    once.step(sum(ks))
    once.check()
    for a, b in zip(many.state(), once.state()):
        assert torch.equal(a, b)
    g = RoesslerChain(*ics, 0.01, exchange=True, graph=True)
    for k in (50, 26, 50, 26, 50):
        g.step(k)
    g.check()
    ref = RoesslerChain(*ics, 0.01, exchange=True)
    ref.step(202)
    ref.check()
    for a, b in zip(g.state(), ref.state()):
        assert torch.equal(a, b)
    for c in (many, once, g, ref):
        c.close()


def test_exchange_at_the_paper_size_equals_fused():
    """N = 2^20, T = 50 steps (the paper's protocol) at the library's
    shape: the whole chain in registers, bit for bit the fused passes."""
    n = 1 << 20
    ics = workloads.roessler_ics(n, 0)
    ref, plan = gpu_run(ics, 0.01, 50)
    ch = RoesslerChain(*ics, 0.01, exchange=True)
    p = ch.plan()
    assert p["exchange"] == 1 and p["waves"] >= 3
    ch.step(50)
    ch.check()
    for a, b in zip((t.cpu().numpy() for t in ch.state()), ref):
        assert np.array_equal(a, b)
    ch.close()


def test_exchange_refuses_chains_it_cannot_hold():
    ics = workloads.roessler_ics(1500, 1)
    with pytest.raises(ChainError):
        RoesslerChain(*ics, 0.01, exchange=True)          # fewer than 3 clusters
    big = workloads.roessler_ics(1 << 22, 1)
    with pytest.raises(ChainError):
        RoesslerChain(*big, 0.01, exchange=True)          # more clusters than the device holds
