"""Continuous-batching job server for chain integrations.

Requests (a chain length, a step count, a precision, a model, an initial
state) arrive over time. The server keeps the admitted jobs' state resident
in HBM and advances all of them in rounds: each round gives every active job
up to `quantum` more steps, with one persistent batch launch per (model,
precision) group, each group on its own stream so their work overlaps on the
device. Between rounds, jobs that finished are retired (energy read back,
memory freed) and waiting jobs are admitted in arrival order while their HBM
footprint and a slot fit. The next round is enqueued before the previous
one's finished jobs are retired, so the device does not idle while the host
does that work. A job's result does not depend on which other jobs share its
rounds: every chain of a batch gives the same bits as the chain run alone.

Failures: a job with a negative step count (or no sites) is rejected on
arrival; a job of zero steps is retired at admission with the energy of its
initial state. Each round's launches report whether a bounded wait for a
neighbour cluster expired (the results of that launch are then invalid); the
jobs of such a launch are stopped at the next round boundary and reported
"failed", without waiting for later rounds that are already queued.

The scheduling policy is independent of the device: `Server` drives an
executor; `GpuExecutor` runs the HIP library, `SimExecutor` replays the same
decisions on a simulated clock (for tests without a GPU).
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

from workloads import Job

FP64, FP32 = 0, 1
PREC_NAMES = {FP64: "fp64", FP32: "fp32_kahan"}
MODEL_NAMES = {0: "quartic", 1: "harmonic"}


@dataclasses.dataclass
class JobResult:
    jid: int
    n: int
    steps: int
    prec: int
    model: int
    arrival: float
    admitted: float = math.nan
    finished: float = math.nan
    energy: float = math.nan
    status: str = "pending"      # done | rejected | cancelled | failed
    waited_for_memory: bool = False  # admission was held back by the HBM budget

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def queue_s(self) -> float:
        return self.admitted - self.arrival

    @property
    def service_s(self) -> float:
        return self.finished - self.admitted


def footprint_bytes(n: int, prec: int) -> int:
    """HBM a job holds while active: state plus its workspace (back buffer,
    FP32 carries, energy partials), 32 bytes per site either way."""
    return 32 * n + 16384


class Server:
    """FIFO admission under an HBM budget and a slot limit; rounds of
    `quantum` steps; pipelined retirement."""

    def __init__(self, executor, hbm_budget: int, max_active: int = 64, quantum: int = 1000):
        if hbm_budget <= 0 or max_active < 1 or quantum < 1:
            raise ValueError("budget, slots and quantum must be positive")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.quantum = int(quantum)
        self.used = 0
        self.peak_used = 0
        self.rounds = 0
        self.admission_log: list[int] = []
        self._cancel: set[int] = set()

    def cancel(self, jid: int) -> None:
        """Drop a job: removed from the queue, or retired at the next round
        boundary if it is running."""
        self._cancel.add(jid)

    def run(self, jobs: list[Job]) -> list[JobResult]:
        ex = self.ex
        results = {j.jid: JobResult(j.jid, j.n, j.steps, j.prec, j.model, j.arrival) for j in jobs}
        arrivals = collections.deque(sorted(jobs, key=lambda j: (j.arrival, j.jid)))
        queue: collections.deque[Job] = collections.deque()
        active: dict[int, dict] = {}        # jid -> {job, slot, left}
        inflight = None                     # (token, [jids finishing in that round])
        ex.start()

        def arrive(now):
            while arrivals and arrivals[0].arrival <= now:
                j = arrivals.popleft()
                if j.steps < 0 or j.n < 1 or footprint_bytes(j.n, j.prec) > self.budget:
                    results[j.jid].status = "rejected"
                    results[j.jid].finished = now
                else:
                    queue.append(j)

        def admit(now):
            while queue:
                j = queue[0]
                if j.jid in self._cancel:
                    queue.popleft()
                    results[j.jid].status = "cancelled"
                    continue
                need = footprint_bytes(j.n, j.prec)
                if len(active) >= self.max_active:
                    break                   # strict FIFO: nobody overtakes the head
                if self.used + need > self.budget:
                    results[j.jid].waited_for_memory = True
                    break
                queue.popleft()
                slot = ex.admit(j)
                self.admission_log.append(j.jid)
                r = results[j.jid]
                r.admitted = ex.now()
                if j.steps == 0:
                    # nothing to integrate: the energy of the initial state
                    r.energy = ex.finish(slot)
                    ex.release(slot)
                    r.finished = ex.now()
                    r.status = "done"
                    continue
                self.used += need
                self.peak_used = max(self.peak_used, self.used)
                active[j.jid] = {"job": j, "slot": slot, "left": j.steps}

        def retire(done_jids, now, stopped=False):
            for jid in done_jids:
                a = active.pop(jid)
                r = results[jid]
                r.finished = now
                if ex.failed(a["slot"]):
                    r.status = "failed"         # a launch it ran in timed out
                elif stopped:
                    r.status = "cancelled"
                else:
                    r.energy = ex.finish(a["slot"])
                    r.status = "done"
                ex.release(a["slot"])
                self.used -= footprint_bytes(a["job"].n, a["job"].prec)

        while arrivals or queue or active or inflight is not None:
            now = ex.now()
            arrive(now)
            admit(now)
            if queue and not active and inflight is None:
                # an empty server always fits the head (oversized jobs were
                # rejected on arrival); never spin
                raise RuntimeError("admission stalled")
            # cancellations of running jobs, and jobs whose launch timed out,
            # take effect at a round boundary
            stop = [jid for jid in active
                    if (jid in self._cancel or ex.failed(active[jid]["slot"])) and
                    (inflight is None or jid not in inflight[1])]
            # launch the next round over every job with steps left
            plan = {}
            for jid, a in active.items():
                if jid in stop or a["left"] == 0:
                    continue
                k = min(self.quantum, a["left"])
                plan[jid] = k
            token = None
            if plan:
                token = ex.launch_round({jid: (active[jid]["slot"], k) for jid, k in plan.items()})
                self.rounds += 1
                for jid, k in plan.items():
                    active[jid]["left"] -= k
            # retire the jobs the previous round finished
            if inflight is not None:
                t_done = ex.wait(inflight[0])
                retire(inflight[1], t_done)
                inflight = None
            if stop:
                retire(stop, ex.now(), stopped=True)
            if token is not None:
                inflight = (token, [jid for jid in plan if active[jid]["left"] == 0])
            elif not active and not queue and arrivals:
                ex.sleep_until(arrivals[0].arrival)
        ex.stop()
        return [results[j.jid] for j in jobs]


def percentiles(xs, qs=(50, 99)):
    xs = sorted(x for x in xs if not math.isnan(x))
    if not xs:
        return {f"p{q}": None for q in qs}
    out = {}
    for q in qs:
        k = (len(xs) - 1) * q / 100.0
        lo, hi = int(math.floor(k)), min(int(math.floor(k)) + 1, len(xs) - 1)
        out[f"p{q}"] = xs[lo] + (xs[hi] - xs[lo]) * (k - lo)
    return out


# ---------------------------------------------------------------------------
# Executors
# ---------------------------------------------------------------------------

class SimExecutor:
    """The server's device side on a simulated clock: a round takes
    (sum of n * steps) / rate seconds after the previous round ends. Rounds
    whose index (from 0) is in `fail_rounds` report a timed-out launch."""

    def __init__(self, rate: float = 4e11, overhead: float = 20e-6, fail_rounds=()):
        self.rate = rate
        self.overhead = overhead
        self.t = 0.0
        self.device_free = 0.0
        self.slots = {}
        self._next = 0
        self.max_concurrent = 0
        self.fail_rounds = set(fail_rounds)
        self._rounds = 0
        self._failed = set()
        self.round_jobs = []          # job ids of each round, in launch order

    def start(self):
        self.t = 0.0

    def stop(self):
        pass

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)

    def admit(self, job):
        self._next += 1
        self.slots[self._next] = {"job": job, "done": 0}
        self.max_concurrent = max(self.max_concurrent, len(self.slots))
        return self._next

    def launch_round(self, work):
        start = max(self.t, self.device_free)
        su = 0
        for slot, k in work.values():
            self.slots[slot]["done"] += k
            su += self.slots[slot]["job"].n * k
        self.device_free = start + self.overhead + su / self.rate
        idx = self._rounds
        self._rounds += 1
        self.round_jobs.append({self.slots[slot]["job"].jid for slot, _ in work.values()})
        return self.device_free, idx, [slot for slot, _ in work.values()]

    def wait(self, token):
        t_done, idx, slots = token
        self.t = max(self.t, t_done)
        if idx in self.fail_rounds:
            self._failed.update(slots)
        return self.t

    def failed(self, slot) -> bool:
        return slot in self._failed

    def finish(self, slot):
        s = self.slots[slot]
        return float(s["done"])        # stands in for the energy: steps run

    def release(self, slot):
        del self.slots[slot]
        self._failed.discard(slot)


class GpuExecutor:
    """Jobs as chains of the HIP library, advanced by persistent batches.

    Rounds run four sites per lane by default, not the library's batch
    default of eight: a round seldom fills the device, and smaller clusters
    end each pass sooner (500 served jobs: p50 latency 0.065 / 0.076 s at
    loads 0.5 / 0.8 against 0.086 / 0.091 s with eight, p99 alike)."""

    def __init__(self, device="cuda", dt: float = 0.01, quantum: int = 1000,
                 max_active: int = 64, hbm_budget: int = 4 << 30, sites_per_lane: int = 4,
                 kdepth: int = 0, keep_state_of=(), spin_limit: int = 0):
        import torch

        from .batch import Batch
        self.torch = torch
        self.Batch = Batch
        self.device = torch.device(device)
        self.dt = dt
        self.quantum = quantum
        self.sites = sites_per_lane
        self.kdepth = kdepth
        self.max_active = max_active
        # clusters the budget can hold, plus the extra clusters a chain's cut
        # can take beyond its share of sites (a partial four-wavefront
        # cluster and up to three one-wavefront ones: at most four per slot)
        tile = Batch.clusters(1 << 30, sites_per_lane, kdepth)
        per_cluster_sites = (1 << 30) / max(tile, 1)
        self.max_clusters = int(hbm_budget / 32 / per_cluster_sites) + 4 * max_active + 8
        self.slots = {}
        self._next = 0
        self.groups = {}              # (model, prec) -> {"batch", "stream", "chains"}
        self.keep_state_of = set(keep_state_of)
        self.kept = {}
        self.t0 = None
        self.retire_stream = torch.cuda.Stream(self.device)
        self.spin_limit = spin_limit   # polls of a bounded wait (0 = library default)
        self._failed = set()           # slots that ran in a launch that timed out

    def start(self):
        self.warm_up()
        self.torch.cuda.synchronize(self.device)
        self.t0 = time.perf_counter()

    def warm_up(self):
        """Before the clock starts: one tiny job of every (model, precision)
        group through admission, a one-step round, the energy and release,
        so the first served jobs do not pay for loading kernels, creating
        streams and building each group's batch."""
        import workloads
        slots = [self.admit(workloads.Job(-1 - i, 0.0, 300, 1, prec, model, 0))
                 for i, (model, prec) in enumerate((m, p) for m in MODEL_NAMES for p in PREC_NAMES)]
        self._wait_round(self.launch_round({s: (s, 1) for s in slots}))
        for s in slots:
            self.finish(s)
            self.release(s)
        self.torch.cuda.synchronize(self.device)

    def stop(self):
        self.torch.cuda.synchronize(self.device)

    def now(self):
        return time.perf_counter() - self.t0

    def sleep_until(self, t):
        d = t - self.now()
        if d > 0:
            time.sleep(d)

    def _group(self, model, prec):
        key = (model, prec)
        if key not in self.groups:
            self.groups[key] = {"stream": self.torch.cuda.Stream(self.device), "batch": None,
                                "members": None}
        return self.groups[key]

    def admit(self, job):
        from .chain import Chain
        import workloads
        torch = self.torch
        g = self._group(job.model, job.prec)
        dtype = torch.float64 if job.prec == FP64 else torch.float32
        with torch.cuda.stream(g["stream"]):
            q0, p0 = workloads.chain_ics_torch(job.n, job.seed, self.device, dtype)
            ch = Chain(q0, p0, self.dt, model=MODEL_NAMES[job.model], prec=PREC_NAMES[job.prec],
                       device=self.device, stream=g["stream"])
        self._next += 1
        self.slots[self._next] = {"job": job, "chain": ch, "group": (job.model, job.prec)}
        return self._next

    def launch_round(self, work):
        torch = self.torch
        by_group = collections.defaultdict(list)
        for slot, k in work.values():
            by_group[self.slots[slot]["group"]].append((slot, k))
        events = []
        for key, items in by_group.items():
            g = self.groups[key]
            members = tuple(s for s, _ in items)
            chains = [self.slots[s]["chain"] for s in members]
            if g["batch"] is None:
                g["batch"] = self.Batch(chains, max_steps=self.quantum, sites_per_lane=self.sites,
                                        kdepth=self.kdepth, max_chains=self.max_active,
                                        max_clusters=self.max_clusters, stream=g["stream"],
                                        spin_limit=self.spin_limit)
            elif g["members"] != members:
                g["batch"].rebind(chains)
            g["members"] = members
            g["batch"].step([k for _, k in items])
            ev = torch.cuda.Event()
            ev.record(g["stream"])
            events.append((ev, g["batch"], g["batch"].last_launch(), members))
        return events

    def _wait_round(self, token):
        from ._lib import CHAIN_ETIMEOUT
        for ev, batch, launch, members in token:
            ev.synchronize()
            if batch.launch_status(launch) == CHAIN_ETIMEOUT:
                self._failed.update(members)

    def wait(self, token):
        """Wait for one round: each group's launch alone (not the rounds
        queued after it), noting the slots of a launch that timed out."""
        self._wait_round(token)
        return self.now()

    def failed(self, slot) -> bool:
        return slot in self._failed

    def finish(self, slot):
        s = self.slots[slot]
        ch = s["chain"]
        # The server has waited for the job's last round, so its state is
        # final; the energy runs on a side stream, not behind the next round.
        ch.set_stream(self.retire_stream)
        e = ch.energy()
        if s["job"].jid in self.keep_state_of:
            cq, cp = ch.carry_tensors()
            self.kept[s["job"].jid] = [t.detach().cpu().clone() for t in
                                       ([ch.q, ch.p] + ([cq, cp] if cq is not None else []))]
        return e

    def release(self, slot):
        s = self.slots.pop(slot)
        self._failed.discard(slot)
        g = self.groups[s["group"]]
        if g["members"] is not None and slot in g["members"]:
            # The group's batch still names this chain: forget its member set
            # (the next round rebinds before it launches) and drop the batch's
            # references, so the chain's device memory is freed now and the
            # HBM actually held stays within what admission counts.
            g["members"] = None
            if g["batch"] is not None:
                g["batch"].chains = []
                g["batch"]._hs = None
        s["chain"].close()
