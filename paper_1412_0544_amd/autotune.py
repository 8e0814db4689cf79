"""Autotuner for the fused kernel's cluster shape, and for the shape of a
persistent batch.

The paper picks its cluster size G from a performance study over G
(Sec. 2.3, Sec. 3.2.1). On the GPU the cluster is 64*S*W sites (S sites per
lane, W wavefronts) and a pass advances k steps, so the study runs over
(S, W, k): each candidate is timed on the device with HIP events over a few
passes of a chain of the requested length, and the fastest is kept. Results
are cached in a JSON file keyed by device, model, precision and the length
bucket (the next power of two), so a later process reuses them.
"""
from __future__ import annotations

import json
import os
import threading

import torch

from .chain import Chain, state_dtype

CACHE_ENV = "CHAIN_RK4_TUNE_CACHE"
_lock = threading.Lock()

SITES = (2, 4, 8, 16)
WAVES = (1, 2, 4, 8)
DEPTHS = (1, 2, 4, 6, 8, 12, 16, 24, 32)


def default_candidates(prec: str = "fp64", model: str = "quartic"):
    """Shapes worth timing: every cluster size at the deeper depths that keep
    at least half of the cluster (the halo of the quartic and harmonic chains
    is 2 sites per step and side); 6 sites per lane is built for the FP64
    quartic and harmonic chains."""
    out = []
    sites = SITES + ((6,) if prec == "fp64" and model in ("quartic", "harmonic") else ())
    for s in sites:
        for w in WAVES:
            for k in (16, 24, 32):
                if 64 * s * w >= 8 * k:
                    out.append((s, w, k))
    return out


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(
        os.path.expanduser("~"), ".cache", "chainrk4", "tune.json")


def bucket(n: int) -> int:
    b = 1
    while b < n:
        b <<= 1
    return b


def key(device, model: str, prec: str, n: int) -> str:
    name = torch.cuda.get_device_name(device).replace(" ", "_")
    return f"{name}|{model}|{prec}|{bucket(n)}"


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(entries: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(entries, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def time_shape(q, p, dt, shape, model="quartic", prec="fp64", steps=48, reps=3, device=None):
    """Best site-updates/s of one (S, W, k) over `reps` runs of `steps` steps."""
    s, w, k = shape
    ch = Chain(q, p, dt, model=model, prec=prec, sites_per_lane=s, waves_per_cluster=w,
               kdepth=k, resident=False, device=device or q.device)
    try:
        ch.step(2 * k)
        best = 0.0
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(ch.stream)
            ch.step(steps)
            b.record(ch.stream)
            b.synchronize()
            best = max(best, q.numel() * steps / (a.elapsed_time(b) / 1e3))
        return best
    finally:
        ch.close()


def tune(n: int, model: str = "quartic", prec: str = "fp64", dt: float = 0.01,
         candidates=None, device="cuda", use_cache: bool = True, steps: int = 48,
         q=None, p=None):
    """Return (best (S, W, k), {shape: SU/s}) for chains of length n."""
    device = torch.device(device)
    k_ = key(device, model, prec, n)
    with _lock:
        if use_cache:
            hit = _load().get(k_)
            if hit:
                return tuple(hit["best"]), {tuple(map(int, s.split(","))): v
                                            for s, v in hit["table"].items()}
    if q is None or p is None:
        g = torch.Generator(device="cpu").manual_seed(12345)
        dtype = state_dtype(prec)
        q = (torch.rand(n, generator=g, dtype=torch.float64) * 2 - 1).to(device, dtype)
        p = (torch.rand(n, generator=g, dtype=torch.float64) * 2 - 1).to(device, dtype)
    table = {}
    for shape in candidates or default_candidates(prec, model):
        table[tuple(shape)] = time_shape(q, p, dt, shape, model, prec, steps=steps, device=device)
    best = max(table, key=table.get)
    with _lock:
        entries = _load()
        entries[k_] = {"best": list(best),
                       "table": {",".join(map(str, s)): v for s, v in table.items()}}
        _store(entries)
    return best, table


BATCH_CANDIDATES = ((4, 16), (4, 24), (4, 32), (8, 16), (8, 24), (8, 32))


def _snapshot(chains):
    out = []
    for c in chains:
        cq, cp = c.carry_tensors()
        out.append([t.clone() for t in (c.q, c.p) + ((cq, cp) if cq is not None else ())])
    return out


def _restore(chains, snap):
    for c, saved in zip(chains, snap):
        cq, cp = c.carry_tensors()
        for dst, src in zip((c.q, c.p) + ((cq, cp) if cq is not None else ()), saved):
            dst.copy_(src)


def batch_key(chains) -> str:
    c = chains[0]
    name = torch.cuda.get_device_name(c.device).replace(" ", "_")
    total = sum(x.q.numel() for x in chains)
    return (f"{name}|batch|{c.desc.model}|{c.desc.prec}|{len(chains)}|{bucket(total)}")


def tune_batch(chains, steps: int = 256, reps: int = 2, candidates=BATCH_CANDIDATES,
               use_cache: bool = True):
    """Return (best (sites_per_lane, kdepth), {shape: SU/s}) for a persistent
    batch over `chains`: each candidate runs `steps` steps `reps` times on the
    chains' own state (saved before and restored after, so the chains end as
    they started), timed on the device."""
    from .batch import Batch
    k_ = batch_key(chains)
    with _lock:
        if use_cache:
            hit = _load().get(k_)
            if hit:
                return tuple(hit["best"]), {tuple(map(int, s.split(","))): v
                                            for s, v in hit["table"].items()}
    total = sum(x.q.numel() for x in chains)
    snap = _snapshot(chains)
    stream = chains[0].stream
    table = {}
    try:
        for s, k in candidates:
            b = Batch(chains, max_steps=steps, sites_per_lane=s, kdepth=k, stream=stream)
            try:
                best = 0.0
                for _ in range(reps + 1):           # the first run warms up
                    a = torch.cuda.Event(enable_timing=True)
                    e = torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    b.step(steps)
                    e.record(stream)
                    b.check()
                    best = max(best, total * steps / (a.elapsed_time(e) / 1e3))
                table[(s, k)] = best
            finally:
                b.close()
    finally:
        _restore(chains, snap)
        torch.cuda.synchronize(chains[0].device)
    best = max(table, key=table.get)
    with _lock:
        entries = _load()
        entries[k_] = {"best": list(best), "table": {",".join(map(str, s)): v
                                                     for s, v in table.items()}}
        _store(entries)
    return best, table
