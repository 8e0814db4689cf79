"""Batches through the C ABI: one persistent launch over many chains.

Every chain of a batch must give the same bits as the chain stepped alone,
for any grid size (one workgroup up to the full device) and any split of the
steps into calls; a sample is checked against the CPU oracle (FP64 bar:
1e-10 max-abs).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1412_0544_amd import Batch, Chain, ChainError
from paper_1412_0544_amd import _lib as L

pytestmark = pytest.mark.gpu
TOL = 1e-10

LENGTHS = [1, 2, 7, 300, 1024, 1025, 2049, 5003, 20011, 65536]


def make_chains(lengths, seeds, prec="fp64", model="quartic", dt=0.01):
    chains = []
    for n, s in zip(lengths, seeds):
        dtype = np.float64 if prec == "fp64" else np.float32
        q0, p0 = workloads.chain_ics(n, s, dtype=dtype)
        chains.append(Chain(q0, p0, dt, model=model, prec=prec))
    return chains


def snapshot(ch):
    out = [ch.q.cpu().numpy().copy(), ch.p.cpu().numpy().copy()]
    cq, cp = ch.carry_tensors()
    if cq is not None:
        out += [cq.cpu().numpy().copy(), cp.cpu().numpy().copy()]
    return out


def solo(n, seed, steps, prec="fp64", model="quartic", dt=0.01):
    dtype = np.float64 if prec == "fp64" else np.float32
    q0, p0 = workloads.chain_ics(n, seed, dtype=dtype)
    ch = Chain(q0, p0, dt, model=model, prec=prec, sites_per_lane=8, kdepth=5, resident=False)
    ch.step(steps)
    out = snapshot(ch)
    ch.close()
    return out


@pytest.mark.parametrize("shape", [(0, 0, 0), (8, 12, 0), (4, 16, 0), (16, 8, 0), (4, 2, 0),
                                   (8, 12, 1), (4, 16, 1), (0, 0, 2), (8, 32, 2), (4, 16, 3)])
def test_batch_matches_solo_bitwise(shape):
    sites, depth, flags = shape
    steps = [37, 0, 1, 100, 5, 2, 64, 13, 3, 24]
    chains = make_chains(LENGTHS, range(10, 20))
    b = Batch(chains, max_steps=100, sites_per_lane=sites, kdepth=depth, flags=flags)
    b.step(steps)
    b.check()
    for ch, n, s, k in zip(chains, LENGTHS, range(10, 20), steps):
        got = snapshot(ch)
        want = solo(n, s, k)
        for x, y in zip(got, want):
            assert np.array_equal(x, y), (n, k, shape)
    b.close()


@pytest.mark.parametrize("prec,flags", [("fp64", 0), ("fp64", L.CHAIN_BATCH_FENCES),
                                        ("fp32_kahan", 0), ("fp64", L.CHAIN_BATCH_WIDE_ONLY)])
def test_narrow_packs_across_chains_match_solo(prec, flags):
    """At 8 sites per lane and depth 32 a wide cluster keeps up to 1916 sites
    and a narrow one up to 380; these lengths end in one, two or three narrow
    clusters (or are nothing else), so packs of four narrow clusters span
    chains, and the differing step counts give the chains different pass
    counts (a pack slot whose chain has no pass left idles)."""
    lengths = [100, 383, 700, 1100, 2116, 4332, 3000, 5000, 257, 9000, 450, 1500, 2300, 4100]
    steps = [64, 1, 0, 33, 96, 5, 32, 17, 2, 64, 31, 65, 95, 40]
    seeds = range(80, 80 + len(lengths))
    narrow = [sum(w == 1 for _, _, w in Batch.layout(n, 8, 32, flags)) for n in lengths]
    if flags & L.CHAIN_BATCH_WIDE_ONLY:
        assert not any(narrow)
    else:
        assert {1, 2, 3} <= set(narrow)
    chains = make_chains(lengths, seeds, prec=prec)
    b = Batch(chains, max_steps=96, sites_per_lane=8, kdepth=32, flags=flags)
    assert b.plan()["narrow_clusters"] == sum(narrow)
    b.step(steps)
    b.check()
    for ch, n, s, k in zip(chains, lengths, seeds, steps):
        got = snapshot(ch)
        want = solo(n, s, k, prec=prec)
        for x, y in zip(got, want):
            assert np.array_equal(x, y), (n, k, prec, flags)
    b.close()


def test_batch_against_oracle():
    steps = [100] * len(LENGTHS)
    chains = make_chains(LENGTHS, range(30, 40))
    b = Batch(chains, max_steps=100)
    b.step(steps)
    b.check()
    e = b.energies()
    for ch, n, s, ek in zip(chains, LENGTHS, range(30, 40), e):
        q0, p0 = workloads.chain_ics(n, s)
        qo, po = oracle.rk4(oracle.QUARTIC, q0, p0, 0.01, 100, threads=8)
        q, p = (t.cpu().numpy() for t in ch.state())
        assert np.abs(q - qo).max() <= TOL and np.abs(p - po).max() <= TOL, n
        eo = oracle.energy(oracle.QUARTIC, qo, po)
        assert abs(ek - eo) <= 1e-12 * abs(eo)


def test_grid_size_and_repeats_do_not_change_bits():
    """Race check: one workgroup, a few, and the full device, repeated."""
    lengths = [300, 5003, 20011, 65536, 100000]
    ref = None
    for grid, flags in ((1, 0), (3, 0), (0, 0), (0, 0), (0, 1), (17, 0), (0, 0), (5, 1), (0, 2),
                        (2, 2)):
        chains = make_chains(lengths, range(50, 55))
        b = Batch(chains, max_steps=60, grid_blocks=grid, flags=flags)
        b.step([60, 41, 60, 33, 60])
        b.check()
        got = [snapshot(c) for c in chains]
        if ref is None:
            ref = got
        else:
            for a, r in zip(got, ref):
                for x, y in zip(a, r):
                    assert np.array_equal(x, y), grid
        b.close()


def test_successive_calls_equal_one_call():
    lengths = [1000, 9000, 33333]
    one = make_chains(lengths, range(60, 63))
    b1 = Batch(one, max_steps=90)
    b1.step(90)
    many = make_chains(lengths, range(60, 63))
    b2 = Batch(many, max_steps=90)
    for k in (1, 2, 30, 57):
        b2.step(k)
    b2.check()
    for x, y in zip(one, many):
        assert torch.equal(x.q, y.q) and torch.equal(x.p, y.p)


@pytest.mark.parametrize("model", ["quartic", "harmonic"])
def test_fp32_batch_matches_solo(model):
    lengths = [64, 1024, 3000, 40000]
    steps = [20, 7, 33, 12]
    chains = make_chains(lengths, range(70, 74), prec="fp32_kahan", model=model)
    b = Batch(chains, max_steps=40)
    b.step(steps)
    b.check()
    for ch, n, s, k in zip(chains, lengths, range(70, 74), steps):
        got = snapshot(ch)
        want = solo(n, s, k, prec="fp32_kahan", model=model)
        for x, y in zip(got, want):
            assert np.array_equal(x, y)


def test_forced_timeout_is_reported_and_kernel_exits():
    """A spin limit of one poll makes items that must wait give up: the call
    reports CHAIN_ETIMEOUT and the launch still finishes. Each launch keeps
    its own timeout word: launch 0 is still reported after launch 1 has been
    queued (its word cleared on the device), and chain_rk4_batch_check
    reports the timeouts of every launch since the previous check, once."""
    chains = make_chains([200000], [80])
    b = Batch(chains, max_steps=400, spin_limit=1)
    b.step(400)
    first = b.last_launch()
    b.step(400)
    assert b.last_launch() == first + 1
    assert b.launch_status(first) == L.CHAIN_ETIMEOUT
    assert b.launch_status(first + 1) == L.CHAIN_ETIMEOUT
    assert b.check_status() == L.CHAIN_ETIMEOUT
    assert b.check_status() == L.CHAIN_OK            # reported once
    b.step(400)
    with pytest.raises(ChainError):
        b.check()
    with pytest.raises(ChainError):
        b.launch_status(b.last_launch() + 1)         # not enqueued
    b.close()
    # the same batch shape with the default limit is fine
    chains = make_chains([200000], [80])
    b = Batch(chains, max_steps=400)
    b.step(400)
    b.check()


def test_batch_rejects_bad_arguments():
    a = make_chains([100], [1], prec="fp64")
    c = make_chains([100], [1], prec="fp32_kahan")
    with pytest.raises(ChainError):
        Batch(a + c, max_steps=10)      # mixed precision
    with pytest.raises(ChainError):
        Batch(a + a, max_steps=10)      # same handle twice
    naive = Chain(np.zeros(10), np.zeros(10), 0.01, method="naive")
    with pytest.raises(ChainError):
        Batch([naive], max_steps=10)
    from paper_1412_0544_amd import tableaus
    tab = Chain(np.zeros(100), np.zeros(100), 0.01, tableau=tableaus.RK4)
    with pytest.raises(ChainError):
        Batch([tab], max_steps=10)      # a Butcher tableau: batches run classical RK4
    b = Batch(a, max_steps=10)
    assert b.last_launch() == -1
    with pytest.raises(ChainError):
        b.step([11])
    with pytest.raises(ChainError):
        b.step([-1])
    with pytest.raises(ChainError):
        b.rebind([tab])
    b.step([0])                         # nothing to do: no launch
    assert b.last_launch() == -1


def test_workload_4096_chains_every_chain():
    """4096 chains, lengths log-uniform in [256, 65536] (seed 4096), ICs per
    chain from seed 1000 + b, dt = 0.01, 100 steps, one launch at the
    library's batch shape: every chain against its solo run (bits, compared on
    the device), and a sample of whole chains against the oracle (1e-10)."""
    lengths = workloads.batch_lengths(4096)
    chains = []
    for i, n in enumerate(lengths):
        q0, p0 = workloads.chain_ics_torch(int(n), 1000 + i, "cuda")
        chains.append(Chain(q0, p0, 0.01))
    b = Batch(chains, max_steps=100)
    b.step(100)
    b.check()
    e = b.energies()
    bad = []
    for i, n in enumerate(lengths):
        q0, p0 = workloads.chain_ics_torch(int(n), 1000 + i, "cuda")
        ref = Chain(q0, p0, 0.01, sites_per_lane=8, kdepth=5, resident=False)
        ref.step(100)
        if not (torch.equal(ref.q, chains[i].q) and torch.equal(ref.p, chains[i].p)):
            bad.append(i)
        ref.close()
    assert not bad, bad[:10]
    rng = np.random.default_rng(1)
    sample = sorted(set(rng.integers(0, 4096, 40).tolist()) | {int(np.argmin(lengths)),
                                                              int(np.argmax(lengths))})
    for i in sample:
        n = int(lengths[i])
        q0, p0 = workloads.chain_ics(n, 1000 + i)
        qo, po = oracle.rk4(oracle.QUARTIC, q0, p0, 0.01, 100, threads=8)
        q, p = (t.cpu().numpy() for t in chains[i].state())
        assert np.abs(q - qo).max() <= TOL and np.abs(p - po).max() <= TOL, i
        eo = oracle.energy(oracle.QUARTIC, qo, po)
        assert abs(e[i] - eo) <= 1e-12 * abs(eo), i
    b.close()
    for c in chains:
        c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_batch_autotuner_leaves_the_chains_as_they_were(prec, tmp_path, monkeypatch):
    """The batch autotuner times its candidates on the chains' own state and
    restores it bit for bit; the shape it returns is one of its candidates,
    and a second call is served from its cache."""
    from paper_1412_0544_amd import autotune
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    dtype = np.float64 if prec == "fp64" else np.float32
    chains = [Chain(*workloads.chain_ics(n, 30 + i, dtype=dtype), 0.01, prec=prec)
              for i, n in enumerate((700, 3000, 20000, 90000))]
    before = [[t.clone() for t in (c.q, c.p) + tuple(x for x in c.carry_tensors()
                                                    if x is not None)] for c in chains]
    best, table = autotune.tune_batch(chains, steps=16, reps=1)
    assert best in autotune.BATCH_CANDIDATES and set(table) == set(autotune.BATCH_CANDIDATES)
    for c, saved in zip(chains, before):
        now = (c.q, c.p) + tuple(x for x in c.carry_tensors() if x is not None)
        for a, b in zip(now, saved):
            assert torch.equal(a, b)
    assert autotune.tune_batch(chains)[0] == best          # cached
    for c in chains:
        c.close()
