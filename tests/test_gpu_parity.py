"""Parity of the HIP path with the CPU oracle, through the C ABI.

FP64 bar: max-abs state error <= 1e-10 after 100 steps (and after 1000 on the
1024-site ring), energy within 1e-12 relative. Every GPU path (fused at any
tile shape and depth, naive, resident) gives the same bits.
"""
import functools
import math

import numpy as np
import pytest
import torch
from scipy.special import ellipj

import oracle
import workloads
from paper_1412_0544_amd import Chain

pytestmark = pytest.mark.gpu
TOL = 1e-10
MODELS = {"quartic": oracle.QUARTIC, "harmonic": oracle.HARMONIC}


def gpu_run(q0, p0, dt, steps, **kw):
    ch = Chain(q0, p0, dt, **kw)
    ch.step(steps)
    e = ch.energy()
    q, p = (t.cpu().numpy() for t in ch.state())
    plan = ch.plan()
    ch.close()
    return q, p, e, plan


@functools.lru_cache(maxsize=None)
def oracle_run(model, n, seed, dt, steps):
    q0, p0 = workloads.chain_ics(n, seed)
    return oracle.rk4(MODELS[model], q0, p0, dt, steps, threads=8)


def maxerr(a, b):
    return float(np.max(np.abs(a - b))) if a.size else 0.0


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 257, 1000, 5003, 20011])
@pytest.mark.parametrize("sites,waves,depth", [(4, 1, 1), (8, 2, 3), (16, 1, 8), (8, 4, 16),
                                               (4, 8, 4), (8, 4, 12), (16, 8, 12), (2, 1, 5),
                                               (2, 4, 16), (8, 4, 32), (6, 4, 32), (6, 1, 7)])
def test_fused_tiled_matches_oracle(n, sites, waves, depth):
    q0, p0 = workloads.chain_ics(n, 1)
    q, p, e, plan = gpu_run(q0, p0, 0.01, 100, sites_per_lane=sites, waves_per_cluster=waves,
                            kdepth=depth, resident=False)
    assert plan["resident"] == 0 and plan["sites_per_lane"] == sites
    assert plan["waves_per_cluster"] == waves
    # a step's edge error reaches 2 sites into the cluster (dq/dt = p is local);
    # the halo covers that, rounded up to a whole 16-byte vector (2 FP64 sites)
    assert plan["halo"] == -(-2 * plan["kdepth"] // 2) * 2
    qo, po = oracle_run("quartic", n, 1, 0.01, 100)
    assert maxerr(q, qo) <= TOL and maxerr(p, po) <= TOL
    eo = oracle.energy(oracle.QUARTIC, qo, po)
    assert abs(e - eo) <= 1e-12 * abs(eo)


@pytest.mark.parametrize("n", [1, 5, 640, 4099])
def test_harmonic_fused_matches_oracle(n):
    q0, p0 = workloads.chain_ics(n, 2)
    qo, po = oracle_run("harmonic", n, 2, 0.05, 100)
    eo = oracle.energy(oracle.HARMONIC, qo, po)
    for sites in (8, 6):
        q, p, e, _ = gpu_run(q0, p0, 0.05, 100, model="harmonic", sites_per_lane=sites,
                             kdepth=4, resident=False)
        assert maxerr(q, qo) <= TOL and maxerr(p, po) <= TOL, sites
        assert abs(e - eo) <= 1e-12 * abs(eo), sites


@pytest.mark.parametrize("n", [1, 2, 3, 100, 1024, 4096])
@pytest.mark.parametrize("model", ["quartic", "harmonic"])
def test_resident_naive_and_tiled_identical_bits(n, model):
    q0, p0 = workloads.chain_ics(n, 3)
    ref = gpu_run(q0, p0, 0.01, 37, model=model, sites_per_lane=8, kdepth=5, resident=False)
    res = gpu_run(q0, p0, 0.01, 37, model=model, resident=True)
    assert res[3]["resident"] == 1
    nav = gpu_run(q0, p0, 0.01, 37, model=model, method="naive")
    for other in (res, nav):
        assert np.array_equal(other[0], ref[0]) and np.array_equal(other[1], ref[1])
    qo, po = oracle_run(model, n, 3, 0.01, 37)
    assert maxerr(ref[0], qo) <= TOL and maxerr(ref[1], po) <= TOL


def test_tile_shapes_and_depths_identical_bits():
    n = 30011
    q0, p0 = workloads.chain_ics(n, 4)
    ref = gpu_run(q0, p0, 0.01, 24, sites_per_lane=4, waves_per_cluster=1, kdepth=1,
                  resident=False)
    for s in (2, 4, 6, 8, 16):
        for w in (1, 2, 4, 8):
            for k in (2, 3, 8, 12, 16, 24, 32):
                got = gpu_run(q0, p0, 0.01, 24, sites_per_lane=s, waves_per_cluster=w, kdepth=k,
                              resident=False)
                assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (s, w, k)
                assert got[2] == ref[2]


@pytest.mark.parametrize("seed", [0, 1])
def test_ring_1024_1000_steps(seed):
    """The 1024-site ring, dt = 0.01, 1000 steps, resident on chip."""
    q0, p0 = workloads.chain_ics(1024, seed)
    q, p, e, plan = gpu_run(q0, p0, 0.01, 1000, resident=True)
    assert plan["resident"] == 1
    q2, p2, e2, plan2 = gpu_run(q0, p0, 0.01, 1000)               # library plan: tiled
    assert plan2["resident"] == 0
    assert np.array_equal(q2, q) and np.array_equal(p2, p) and e2 == e
    qo, po = oracle_run("quartic", 1024, seed, 0.01, 1000)
    assert maxerr(q, qo) <= TOL and maxerr(p, po) <= TOL
    eo = oracle.energy(oracle.QUARTIC, qo, po)
    assert abs(e - eo) <= 1e-12 * abs(eo)


@pytest.mark.parametrize("steps", [0, 1, 2, 3, 5, 8, 9, 17])
@pytest.mark.parametrize("depth", [1, 4])
def test_step_counts_and_pass_parity(steps, depth):
    """Odd and even pass counts, split passes and the copy-back path."""
    n = 3001
    q0, p0 = workloads.chain_ics(n, 5)
    q, p, _, _ = gpu_run(q0, p0, 0.01, steps, sites_per_lane=8, kdepth=depth, resident=False)
    qo, po = oracle_run("quartic", n, 5, 0.01, steps)
    assert maxerr(q, qo) <= TOL and maxerr(p, po) <= TOL
    if steps == 0:
        assert np.array_equal(q, q0) and np.array_equal(p, p0)


def test_split_calls_equal_one_call():
    n = 7000
    q0, p0 = workloads.chain_ics(n, 6)
    one = gpu_run(q0, p0, 0.01, 60, sites_per_lane=8, kdepth=8, resident=False)
    ch = Chain(q0, p0, 0.01, sites_per_lane=8, kdepth=8, resident=False)
    for k in (1, 7, 13, 39):
        ch.step(k)
    q, p = (t.cpu().numpy() for t in ch.state())
    ch.close()
    assert np.array_equal(q, one[0]) and np.array_equal(p, one[1])


def test_time_reversal_bitwise():
    n = 2050
    q0, p0 = workloads.chain_ics(n, 7)
    a = gpu_run(q0, -p0, 0.01, 40, sites_per_lane=8, kdepth=4, resident=False)
    b = gpu_run(q0, p0, -0.01, 40, sites_per_lane=16, waves_per_cluster=4, kdepth=8,
                resident=False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], -b[1])


def test_shift_and_reflection_bitwise():
    n = 5000
    q0, p0 = workloads.chain_ics(n, 8)
    kw = dict(sites_per_lane=8, kdepth=4, resident=False)
    base = gpu_run(q0, p0, 0.01, 32, **kw)
    for s in (1, 77, 4999):
        sh = gpu_run(np.roll(q0, s), np.roll(p0, s), 0.01, 32, **kw)
        assert np.array_equal(sh[0], np.roll(base[0], s)) and np.array_equal(sh[1], np.roll(base[1], s))
    rf = gpu_run(q0[::-1].copy(), p0[::-1].copy(), 0.01, 32, **kw)
    assert np.array_equal(rf[0][::-1], base[0]) and np.array_equal(rf[1][::-1], base[1])


def test_graph_replays_match_eager():
    n = 9000
    q0, p0 = workloads.chain_ics(n, 9)
    eager = Chain(q0, p0, 0.01, sites_per_lane=8, kdepth=4, resident=False)
    graph = Chain(q0, p0, 0.01, sites_per_lane=8, kdepth=4, resident=False, graph=True)
    for rep in range(4):
        eager.step(10)
        graph.step(10)
        torch.cuda.synchronize()
        assert torch.equal(eager.q, graph.q) and torch.equal(eager.p, graph.p), rep
        _ = eager.energy()
    eager.close()
    graph.close()


@pytest.mark.parametrize("n,shape", [(1 << 17, (4, 1, 32)), ((1 << 18) + 77, (6, 1, 32)),
                                     (1 << 19, (6, 1, 32)), (1 << 21, (6, 4, 32))])
def test_library_plans_of_chains_that_fill_the_chip_once(n, shape):
    """The default plans of chains that fill the chip about once (the rows
    picked by the granularity study): every site after 100 steps against the
    oracle's whole-ring run, and the energy."""
    import os
    q0, p0 = workloads.chain_ics(n, 6)
    q, p, e, plan = gpu_run(q0, p0, 0.01, 100)
    assert (plan["sites_per_lane"], plan["waves_per_cluster"], plan["kdepth"]) == shape
    threads = max(1, min(16, os.cpu_count() or 1))
    qo, po = oracle.rk4(oracle.QUARTIC, q0, p0, 0.01, 100, threads=threads)
    assert maxerr(q, qo) <= TOL and maxerr(p, po) <= TOL
    eo = oracle.energy(oracle.QUARTIC, qo, po)
    assert abs(e - eo) <= 1e-12 * abs(eo)


FULL = 1 << 24


@pytest.fixture(scope="module")
def full_ics():
    return workloads.chain_ics(FULL, 0)


def test_full_size_sampled_sites(full_ics):
    """N = 2^24, dt = 0.01, 100 steps, default fused plan: sampled sites vs the
    oracle, each from its own light cone."""
    q0, p0 = full_ics
    q, p, e, plan = gpu_run(q0, p0, 0.01, 100)
    assert plan["resident"] == 0
    tile = plan["tile"]
    rng = np.random.default_rng(0)
    sites = np.unique(np.concatenate([
        [0, 1, FULL - 1, FULL - 2, tile - 1, tile, 2 * tile - 1, 2 * tile],
        (np.arange(1, 9) * 1_999_993) % FULL,
        rng.integers(0, FULL, 16)]))
    qs, ps = oracle.rk4_sites(oracle.QUARTIC, q0, p0, 0.01, 100, sites)
    assert maxerr(q[sites], qs) <= TOL and maxerr(p[sites], ps) <= TOL
    assert np.all(np.isfinite(q)) and np.all(np.isfinite(p))


def test_full_size_every_site_against_the_oracle(full_ics):
    """N = 2^24, dt = 0.01, 100 steps, the default fused plan (the benchmark's
    launch configuration): every one of the 2^24 sites against the oracle's
    whole-ring run (Sec. 2.3: every cluster's kept sites are the exact
    standard RK4 result), and the energy."""
    import os
    q0, p0 = full_ics
    q, p, e, plan = gpu_run(q0, p0, 0.01, 100)
    assert plan["resident"] == 0 and plan["waves"] > 8000
    threads = max(1, min(16, os.cpu_count() or 1))
    qo, po = oracle.rk4(oracle.QUARTIC, q0, p0, 0.01, 100, threads=threads)
    assert maxerr(q, qo) <= TOL and maxerr(p, po) <= TOL
    eo = oracle.energy(oracle.QUARTIC, qo, po)
    assert abs(e - eo) <= 1e-12 * abs(eo)


def test_full_size_every_tuned_shape_identical_bits(full_ics):
    """Every cluster shape the autotuner may pick for the benchmark gives the
    same bits at N = 2^24 as the default plan (checked against the oracle
    above)."""
    from paper_1412_0544_amd import autotune
    q0, p0 = full_ics
    qd = torch.from_numpy(q0).cuda()
    pd = torch.from_numpy(p0).cuda()
    ref = Chain(qd, pd, 0.01)
    ref.step(30)
    for s, w, k in autotune.default_candidates():
        ch = Chain(qd, pd, 0.01, sites_per_lane=s, waves_per_cluster=w, kdepth=k, resident=False)
        ch.step(30)
        torch.cuda.synchronize()
        assert torch.equal(ch.q, ref.q) and torch.equal(ch.p, ref.p), (s, w, k)
        ch.close()
    ref.close()


def test_full_size_pi_mode_closed_form():
    """q_i = (-1)^i A stays an exact alternation (any halo or tile-edge error
    breaks it) and follows A cn(Omega t | m) with Omega^2 = 1 + 17 A^2."""
    A, dt, steps = 0.8, 0.01, 1000
    q0, p0 = workloads.mode_ics(FULL, "pi", A)
    q, p, e, _ = gpu_run(q0, p0, dt, steps)
    s = np.where(np.arange(FULL) % 2 == 0, 1.0, -1.0)
    assert np.array_equal(q * s, np.full(FULL, q[0]))
    assert np.array_equal(p * s, np.full(FULL, p[0]))
    om = math.sqrt(1 + 17 * A * A)
    m = 17 * A * A / (2 * om * om)
    sn, cn, dn, _ = ellipj(om * steps * dt, m)
    assert abs(q[0] - A * cn) < 2e-6
    assert abs(e - FULL * (A * A / 2 + 17 * A ** 4 / 4)) <= 1e-6 * e


# --------------------------------------------------------------------------
# FP32 state with compensated update (stated accuracy against the FP64
# oracle started from the FP32-rounded initial state).
# --------------------------------------------------------------------------

# Max-abs error against the FP64 oracle after 100 steps of dt = 0.01, over
# every site of chains of up to 2^16 sites (the runs are bitwise
# reproducible). Measured, compensated with FP32 / FP64 carries: 2.4e-8 /
# 2.0e-8 at N <= 3, 1.6e-7 / 1.8e-7 at N = 1000, 1.9e-7 / 2.0e-7 at 20011 and
# 2.4e-7 / 2.3e-7 at 2^16 (the largest error grows slowly with the number of
# sites); plain FP32 1.5e-6 at N = 1000 and 3.4e-6 at 20011 and 2^16. The bar
# sits 2x above the compensated forms and 3x below plain FP32 at N >= 1000,
# so it tells them apart by itself (test_plain_fp32_control checks that the
# control fails it).
FP32_TOL_100 = 5e-7


@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32_kahan64"])
@pytest.mark.parametrize("n", [1, 3, 1000, 20011])
def test_fp32_kahan_error_bound(n, prec):
    q0, p0 = workloads.chain_ics(n, 10, dtype=np.float32)
    ch = Chain(q0, p0, 0.01, prec=prec, sites_per_lane=16, kdepth=4, resident=False)
    ch.step(100)
    cq, cp = ch.carry_tensors()
    q = ch.q.double() - cq.double()
    p = ch.p.double() - cp.double()
    e = ch.energy()
    q, p = q.cpu().numpy(), p.cpu().numpy()
    ch.close()
    qo, po = oracle.rk4(oracle.QUARTIC, q0.astype(np.float64), p0.astype(np.float64), 0.01, 100)
    assert maxerr(q, qo) <= FP32_TOL_100 and maxerr(p, po) <= FP32_TOL_100
    eo = oracle.energy(oracle.QUARTIC, qo, po)
    assert abs(e - eo) <= 1e-5 * abs(eo)


def test_fp32_paths_identical_bits():
    n = 4000
    q0, p0 = workloads.chain_ics(n, 11, dtype=np.float32)
    outs = []
    for kw in (dict(sites_per_lane=16, kdepth=4, resident=False),
               dict(sites_per_lane=8, kdepth=7, waves_per_cluster=1, resident=False),
               dict(sites_per_lane=4, kdepth=12, waves_per_cluster=8, resident=False),
               dict(sites_per_lane=16, kdepth=8, waves_per_cluster=4, resident=False),
               dict(sites_per_lane=2, kdepth=5, waves_per_cluster=2),
               dict(sites_per_lane=2, kdepth=9, waves_per_cluster=1),
               dict(method="naive"), dict(resident=True), dict()):
        ch = Chain(q0, p0, 0.01, prec="fp32_kahan", **kw)
        ch.step(30)
        cq, cp = ch.carry_tensors()
        outs.append([t.cpu().numpy().copy() for t in (ch.q, ch.p, cq, cp)])
        ch.close()
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_fp32_fp64_carry_paths_identical_bits():
    """FP32 state with FP64 carries: every tiled shape and the per-stage
    method give the same bits, carries included."""
    n = 4000
    q0, p0 = workloads.chain_ics(n, 12, dtype=np.float32)
    outs = []
    for kw in (dict(sites_per_lane=16, kdepth=4), dict(sites_per_lane=8, kdepth=7, waves_per_cluster=1),
               dict(sites_per_lane=4, kdepth=12, waves_per_cluster=8),
               dict(sites_per_lane=16, kdepth=8, waves_per_cluster=4),
               dict(sites_per_lane=2, kdepth=5, waves_per_cluster=2),
               dict(method="naive"), dict()):
        ch = Chain(q0, p0, 0.01, prec="fp32_kahan64", **kw)
        ch.step(30)
        cq, cp = ch.carry_tensors()
        assert cq.dtype == torch.float64
        outs.append([t.cpu().numpy().copy() for t in (ch.q, ch.p, cq, cp)])
        ch.close()
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_plain_fp32_control():
    """Plain FP32 (no compensation): every tiled shape and the per-stage
    method give the same bits; its 100-step error stays within 1e-4 of the
    FP64 oracle and is at least 4x the compensated form's (N = 2^16)."""
    n = 1 << 16
    q0, p0 = workloads.chain_ics(n, 14, dtype=np.float32)
    outs = []
    for kw in (dict(sites_per_lane=16, kdepth=4), dict(sites_per_lane=8, kdepth=7, waves_per_cluster=1),
               dict(sites_per_lane=16, kdepth=32, waves_per_cluster=4),
               dict(sites_per_lane=2, kdepth=5, waves_per_cluster=2), dict(method="naive"), dict()):
        ch = Chain(q0, p0, 0.01, prec="fp32", **kw)
        ch.step(100)
        assert ch.carry_tensors() == (None, None)
        outs.append([t.cpu().numpy().copy() for t in (ch.q, ch.p)])
        ch.close()
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)
    qs, ps = oracle.rk4(oracle.QUARTIC, q0.astype(np.float64), p0.astype(np.float64), 0.01, 100,
                        threads=8)
    plain = max(maxerr(outs[0][0], qs), maxerr(outs[0][1], ps))
    ch = Chain(q0, p0, 0.01, prec="fp32_kahan")
    ch.step(100)
    cq, cp = ch.carry_tensors()
    q = (ch.q.double() - cq.double()).cpu().numpy()
    p = (ch.p.double() - cp.double()).cpu().numpy()
    ch.close()
    comp = max(maxerr(q, qs), maxerr(p, ps))
    assert plain <= 1e-4 and comp * 4 <= plain, (plain, comp)
    assert comp <= FP32_TOL_100 < plain, (plain, comp)


@pytest.mark.parametrize("model", ["harmonic", "quartic_nnn"])
def test_fp64_carry_other_models(model):
    n, steps = 3001, 60
    q0, p0 = workloads.chain_ics(n, 13, dtype=np.float32)
    ch = Chain(q0, p0, 0.01, model=model, prec="fp32_kahan64")
    ch.step(steps)
    cq, cp = ch.carry_tensors()
    q = (ch.q.double() - cq).cpu().numpy()
    p = (ch.p.double() - cp).cpu().numpy()
    e = ch.energy()
    ch.close()
    mid = {"harmonic": oracle.HARMONIC, "quartic_nnn": oracle.QUARTIC_NNN}[model]
    qo, po = oracle.rk4(mid, q0.astype(np.float64), p0.astype(np.float64), 0.01, steps)
    assert maxerr(q, qo) <= FP32_TOL_100 and maxerr(p, po) <= FP32_TOL_100
    eo = oracle.energy(mid, qo, po)
    assert abs(e - eo) <= 1e-5 * abs(eo)


def test_chain_longer_than_two_to_the_31():
    """N = 2^31 + 12345 sites (34 GB of state): 64-bit site indexing in every
    kernel of the default plan. Sampled sites, including those around 2^31
    and both ring ends, against the oracle on windows cut from the same
    initial state (whose values are drawn per site index)."""
    n, steps = (1 << 31) + 12345, 10
    q0, p0 = workloads.chain_ics_torch(n, 9, "cuda")
    ch = Chain(q0, p0, 0.01)
    del q0, p0
    torch.cuda.empty_cache()
    ch.step(steps)
    e = ch.energy()
    assert np.isfinite(e)
    r = 4 * steps
    sites = [0, 1, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, n - 2, n - 1, 987654321]
    idx = torch.tensor(sites, device="cuda")
    qg, pg = ch.q[idx].cpu().numpy(), ch.p[idx].cpu().numpy()
    ch.close()
    for k, i in enumerate(sites):
        w = (np.arange(i - r, i + r + 1) % n).astype(np.uint64)
        qw = 2.0 * workloads.uniform01(9, 2 * w) - 1.0
        pw = 2.0 * workloads.uniform01(9, 2 * w + 1) - 1.0
        qo, po = oracle.rk4(oracle.QUARTIC, qw, pw, 0.01, steps)
        assert abs(qg[k] - qo[r]) <= TOL and abs(pg[k] - po[r]) <= TOL, i
