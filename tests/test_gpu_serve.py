"""Continuous-batching server on the GPU: jobs of mixed length, step count,
precision and model arrive while others run; each job's final state is the
same bits as the job run alone, and FP64 jobs match the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1412_0544_amd import Batch, Chain
from paper_1412_0544_amd.serve import GpuExecutor, Server, MODEL_NAMES, PREC_NAMES

pytestmark = pytest.mark.gpu


def alone(job, dt=0.01):
    dtype = torch.float64 if job.prec == 0 else torch.float32
    q0, p0 = workloads.chain_ics_torch(job.n, job.seed, "cuda", dtype)
    ch = Chain(q0, p0, dt, model=MODEL_NAMES[job.model], prec=PREC_NAMES[job.prec])
    ch.step(job.steps)
    e = ch.energy()
    cq, cp = ch.carry_tensors()
    out = [t.cpu().clone() for t in ([ch.q, ch.p] + ([cq, cp] if cq is not None else []))]
    ch.close()
    return out, e


def test_device_ic_generator_matches_host():
    for n, seed in [(1, 0), (4097, 9), (100000, 2**40 + 3)]:
        q, p = workloads.chain_ics(n, seed)
        qt, pt = workloads.chain_ics_torch(n, seed, "cuda")
        assert np.array_equal(q, qt.cpu().numpy()) and np.array_equal(p, pt.cpu().numpy())


def test_served_jobs_equal_alone_runs():
    jobs = workloads.served_jobs(14, rate=400.0, seed=11, n_lo=1000, n_hi=150_000,
                                 steps_lo=200, steps_hi=2500)
    keep = [j.jid for j in jobs]
    ex = GpuExecutor(quantum=400, max_active=5, hbm_budget=64 << 20, keep_state_of=keep)
    srv = Server(ex, hbm_budget=64 << 20, max_active=5, quantum=400)
    res = srv.run(jobs)
    assert all(r.status == "done" for r in res)
    assert srv.peak_used <= 64 << 20
    assert srv.rounds >= 2
    # every job was released: no batch still holds a retired chain
    assert all(g["batch"] is None or not g["batch"].chains for g in ex.groups.values())
    for j, r in zip(jobs, res):
        want, e = alone(j)
        got = ex.kept[j.jid]
        for a, b in zip(got, want):
            assert torch.equal(a, b), j
        assert r.energy == e
    # FP64 jobs against the oracle, sampled sites from their light cones
    for j in jobs:
        if j.prec != 0:
            continue
        q0, p0 = workloads.chain_ics(j.n, j.seed)
        sites = np.array([0, j.n // 3, j.n - 1])
        qs, ps = oracle.rk4_sites(j.model, q0, p0, 0.01, j.steps, sites, threads=8) \
            if 8 * j.steps + 1 < j.n else (None, None)
        if qs is None:
            qo, po = oracle.rk4(j.model, q0, p0, 0.01, j.steps, threads=8)
            qs, ps = qo[sites], po[sites]
        got = ex.kept[j.jid]
        assert np.abs(got[0].numpy()[sites] - qs).max() <= 1e-10
        assert np.abs(got[1].numpy()[sites] - ps).max() <= 1e-10


def test_batch_rebind_to_other_chains():
    a = [Chain(*workloads.chain_ics(n, 90 + i), 0.01) for i, n in enumerate([3000, 70000])]
    b_set = [Chain(*workloads.chain_ics(n, 95 + i), 0.01) for i, n in enumerate([500, 20000, 9000])]
    cap = sum(Batch.clusters(c.q.numel()) for c in a + b_set)
    b = Batch(a, max_steps=50, max_chains=4, max_clusters=cap)
    b.step([50, 40])
    b.rebind(b_set)
    b.step([33, 50, 7])
    b.check()
    for ch, n, seed, k in [(a[0], 3000, 90, 50), (a[1], 70000, 91, 40), (b_set[0], 500, 95, 33),
                           (b_set[1], 20000, 96, 50), (b_set[2], 9000, 97, 7)]:
        ref = Chain(*workloads.chain_ics(n, seed), 0.01, sites_per_lane=4, kdepth=3, resident=False)
        ref.step(k)
        assert torch.equal(ref.q, ch.q) and torch.equal(ref.p, ch.p)
    too_many = a + b_set
    from paper_1412_0544_amd import ChainError
    with pytest.raises(ChainError):
        b.rebind(too_many)


def test_jobs_of_timed_out_launches_fail_and_the_rest_are_exact():
    """With a spin limit of one poll, launches whose items had to wait for a
    neighbour report a timeout: their jobs end "failed" (the server reads
    each round's own timeout word while the next round runs), the server
    still finishes, and every job reported "done" is the same bits as the job
    run alone."""
    jobs = workloads.served_jobs(10, rate=2000.0, seed=17, n_lo=20_000, n_hi=300_000,
                                 steps_lo=300, steps_hi=1500)
    keep = [j.jid for j in jobs]
    ex = GpuExecutor(quantum=300, max_active=4, hbm_budget=256 << 20, keep_state_of=keep,
                     spin_limit=1)
    srv = Server(ex, hbm_budget=256 << 20, max_active=4, quantum=300)
    res = srv.run(jobs)
    assert all(r.status in ("done", "failed") for r in res)
    assert any(r.status == "failed" for r in res)
    assert srv.used == 0 and not ex.slots
    for j, r in zip(jobs, res):
        if r.status == "done":
            want, e = alone(j)
            for a, b in zip(ex.kept[j.jid], want):
                assert torch.equal(a, b), j
            assert r.energy == e
