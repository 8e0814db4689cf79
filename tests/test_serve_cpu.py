"""The serving policy on a simulated clock (no GPU): admission under the HBM
budget and slot limit, strict arrival order, rejection, cancellation, and
latency accounting."""
import math

import pytest

import workloads
from paper_1412_0544_amd.serve import (Server, SimExecutor, footprint_bytes, percentiles)
from workloads import Job


def jobs_small(count=40, rate=50.0, seed=3):
    return workloads.served_jobs(count, rate, seed=seed, n_lo=1000, n_hi=200_000,
                                 steps_lo=100, steps_hi=5000)


def test_all_jobs_complete_with_their_steps():
    jobs = jobs_small()
    ex = SimExecutor(rate=1e9)
    srv = Server(ex, hbm_budget=64 << 20, max_active=8, quantum=700)
    res = srv.run(jobs)
    for j, r in zip(jobs, res):
        assert r.status == "done"
        assert r.energy == j.steps          # the simulated executor reports steps run
        assert r.finished >= r.admitted >= r.arrival
        assert r.latency > 0
    assert not ex.slots                      # everything released


def test_budget_and_slots_are_never_exceeded():
    jobs = jobs_small(80, rate=500.0)
    ex = SimExecutor(rate=5e8)
    budget = 20 << 20
    srv = Server(ex, hbm_budget=budget, max_active=5, quantum=300)
    srv.run(jobs)
    assert srv.peak_used <= budget
    assert ex.max_concurrent <= 5
    assert srv.used == 0


def test_admission_is_in_arrival_order():
    jobs = jobs_small(60, rate=1000.0)
    srv = Server(SimExecutor(rate=2e8), hbm_budget=16 << 20, max_active=4, quantum=500)
    srv.run(jobs)
    order = sorted(jobs, key=lambda j: (j.arrival, j.jid))
    assert srv.admission_log == [j.jid for j in order]


def test_head_of_line_is_not_overtaken():
    """A large job waiting for memory at the head of the queue is not
    overtaken by small jobs that would fit (no starvation)."""
    blocker = Job(1, 0.0, 300_000, 3000, 0, 0, 2)
    big = Job(0, 0.0005, 400_000, 200, 0, 0, 1)
    small = [Job(2 + i, 0.001 * (i + 1), 1000, 100, 0, 0, 3 + i) for i in range(5)]
    budget = footprint_bytes(400_000, 0) + footprint_bytes(1000, 0) * 2
    srv = Server(SimExecutor(rate=1e9), hbm_budget=budget, max_active=8, quantum=100)
    res = srv.run([blocker, big] + small)
    assert srv.admission_log == [1, 0, 2, 3, 4, 5, 6]
    assert all(r.status == "done" for r in res)
    # the small jobs waited behind the big one
    assert all(r.admitted >= res[1].admitted for r in res[2:])


def test_oversized_job_is_rejected():
    jobs = [Job(0, 0.0, 10_000_000, 100, 0, 0, 1), Job(1, 0.0, 1000, 100, 0, 0, 2)]
    srv = Server(SimExecutor(), hbm_budget=1 << 20, max_active=4, quantum=100)
    res = srv.run(jobs)
    assert res[0].status == "rejected" and res[1].status == "done"


def test_cancel_queued_and_running_jobs():
    jobs = [Job(i, 0.0, 100_000, 20_000, 0, 0, i) for i in range(4)]
    ex = SimExecutor(rate=1e9)
    srv = Server(ex, hbm_budget=footprint_bytes(100_000, 0) * 2, max_active=2, quantum=1000)
    srv.cancel(0)   # will be running
    srv.cancel(3)   # still queued when it reaches the head
    res = srv.run(jobs)
    assert res[0].status == "cancelled" and res[3].status == "cancelled"
    assert res[1].status == "done" and res[2].status == "done"
    assert not ex.slots and srv.used == 0


def test_throughput_and_percentiles():
    jobs = jobs_small(50, rate=20.0)
    ex = SimExecutor(rate=1e9, overhead=0.0)
    res = Server(ex, hbm_budget=1 << 30, max_active=64, quantum=1000).run(jobs)
    makespan = max(r.finished for r in res) - min(r.arrival for r in res)
    su = sum(r.n * r.steps for r in res)
    assert su / makespan <= 1e9 * (1 + 1e-9)
    p = percentiles([r.latency for r in res])
    assert 0 < p["p50"] <= p["p99"]
    assert math.isnan(percentiles([])["p50"] or math.nan)


def test_bad_configuration():
    with pytest.raises(ValueError):
        Server(SimExecutor(), hbm_budget=0)


@pytest.mark.timeout(30)
def test_zero_step_job_is_retired_at_admission():
    """A job of zero steps finishes at once with the energy of its initial
    state (the simulated executor reports the steps run: 0) and the server
    does not wait for a round that will never carry it."""
    jobs = [Job(0, 0.0, 5000, 0, 0, 0, 1), Job(1, 0.0, 2000, 300, 1, 1, 2),
            Job(2, 0.01, 3000, 0, 1, 0, 3)]
    ex = SimExecutor(rate=1e9)
    srv = Server(ex, hbm_budget=1 << 30, max_active=4, quantum=100)
    res = srv.run(jobs)
    assert [r.status for r in res] == ["done", "done", "done"]
    assert res[0].energy == 0.0 and res[2].energy == 0.0 and res[1].energy == 300
    assert res[0].finished >= res[0].admitted >= res[0].arrival
    assert not ex.slots and srv.used == 0


@pytest.mark.timeout(30)
def test_negative_steps_and_empty_chains_are_rejected():
    jobs = [Job(0, 0.0, 5000, -1, 0, 0, 1), Job(1, 0.0, 0, 10, 0, 0, 2),
            Job(2, 0.0, 1000, 10, 0, 0, 3)]
    srv = Server(SimExecutor(rate=1e9), hbm_budget=1 << 30, max_active=4, quantum=100)
    res = srv.run(jobs)
    assert [r.status for r in res] == ["rejected", "rejected", "done"]


@pytest.mark.timeout(30)
@pytest.mark.parametrize("bad_round", [0, 3])
def test_jobs_of_a_timed_out_launch_fail_and_the_rest_complete(bad_round):
    """A launch whose bounded wait expired makes its jobs' results invalid:
    they end "failed" (stopped at the next round boundary, or at their end),
    every other job completes, and all memory is released."""
    jobs = [Job(i, 0.002 * i, 20_000 + 1000 * i, 700 * (1 + i % 5), 0, 0, i) for i in range(12)]
    ex = SimExecutor(rate=1e9, fail_rounds={bad_round})
    srv = Server(ex, hbm_budget=1 << 30, max_active=4, quantum=500)
    res = srv.run(jobs)
    failed = [r for r in res if r.status == "failed"]
    assert failed and all(math.isnan(r.energy) for r in failed)
    assert all(r.status in ("done", "failed") for r in res)
    for r in res:
        if r.status == "done":
            assert r.energy == r.steps
    assert not ex.slots and srv.used == 0
    # exactly the jobs of the failing round failed
    assert {r.jid for r in failed} == ex.round_jobs[bad_round]


def test_memory_waits_are_recorded():
    blocker = Job(1, 0.0, 300_000, 3000, 0, 0, 2)
    big = Job(0, 0.0005, 400_000, 200, 0, 0, 1)
    budget = footprint_bytes(400_000, 0) + footprint_bytes(1000, 0) * 2
    res = Server(SimExecutor(rate=1e9), hbm_budget=budget, max_active=8,
                 quantum=100).run([blocker, big])
    assert res[1].waited_for_memory and not res[0].waited_for_memory


class _Stream:
    cuda_stream = 0


class _Event:
    def record(self, stream):
        pass

    def synchronize(self):
        pass


class _Chain:
    def __init__(self, q0, p0, dt, **kw):
        self.q, self.p, self.handle, self.closed = q0, p0, object(), False

    def set_stream(self, stream):
        pass

    def energy(self):
        return 1.0

    def carry_tensors(self):
        return None, None

    def close(self):
        self.closed = True


class _Batch:
    """Stands in for the library batch: checks the executor's calls."""
    timed_out = set()       # launch ids that report a timeout
    launched = []

    def __init__(self, chains, **kw):
        self.chains, self._hs, self.n = list(chains), object(), 0

    @staticmethod
    def clusters(n, sites_per_lane=0, kdepth=0):
        return 1

    def rebind(self, chains):
        self.chains, self._hs = list(chains), object()
        return self

    def step(self, ks):
        assert len(ks) == len(self.chains) and all(not c.closed for c in self.chains)
        self.n += 1
        _Batch.launched.append(self)

    def last_launch(self):
        return self.n - 1

    def launch_status(self, launch):
        return -6 if (id(self), launch) in _Batch.timed_out else 0


@pytest.fixture
def executor_with_stand_ins(monkeypatch):
    """GpuExecutor with its device objects replaced, to check its
    bookkeeping (warm-up, rounds, retire, release, timeouts) on the CPU."""
    import contextlib
    import torch
    from paper_1412_0544_amd import batch as batch_mod, chain as chain_mod, serve
    monkeypatch.setattr(torch.cuda, "Stream", lambda *a, **k: _Stream())
    monkeypatch.setattr(torch.cuda, "Event", lambda *a, **k: _Event())
    monkeypatch.setattr(torch.cuda, "stream", lambda s: contextlib.nullcontext())
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(workloads, "chain_ics_torch",
                        lambda n, seed, dev, dtype=torch.float64: (torch.zeros(n), torch.zeros(n)))
    monkeypatch.setattr(chain_mod, "Chain", _Chain)
    monkeypatch.setattr(batch_mod, "Batch", _Batch)
    _Batch.timed_out, _Batch.launched = set(), []
    return serve.GpuExecutor


@pytest.mark.timeout(60)
def test_gpu_executor_bookkeeping(executor_with_stand_ins):
    ex = executor_with_stand_ins(device="cpu", quantum=400, max_active=5, hbm_budget=64 << 20)
    jobs = workloads.served_jobs(14, rate=400.0, seed=11, n_lo=1000, n_hi=150_000,
                                 steps_lo=200, steps_hi=2500)
    srv = Server(ex, hbm_budget=64 << 20, max_active=5, quantum=400)
    res = srv.run(jobs)
    assert all(r.status == "done" for r in res)
    assert srv.used == 0 and not ex.slots
    # retired chains are dropped from the batches that ran them
    assert all(g["batch"] is None or not g["batch"].chains for g in ex.groups.values())


@pytest.mark.timeout(60)
def test_gpu_executor_fails_the_jobs_of_a_timed_out_launch(executor_with_stand_ins):
    ex = executor_with_stand_ins(device="cpu", quantum=300, max_active=4, hbm_budget=64 << 20)
    jobs = [Job(i, 0.0, 5000, 900, 0, 0, i) for i in range(3)]
    srv = Server(ex, hbm_budget=64 << 20, max_active=4, quantum=300)
    orig = _Batch.step

    def step_and_time_out(self, ks):
        orig(self, ks)
        if self.n == 2:                  # the second launch of the group times out
            _Batch.timed_out.add((id(self), self.n - 1))
    _Batch.step = step_and_time_out
    try:
        res = srv.run(jobs)
    finally:
        _Batch.step = orig
    assert [r.status for r in res] == ["failed"] * 3
    assert srv.used == 0 and not ex.slots
