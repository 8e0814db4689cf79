"""Seeded synthetic inputs for the chain RK4 workloads.

This module is shared by the CPU oracle side and the GPU side. It holds no
part of the integration method: it only produces the initial conditions, chain
lengths, step counts and arrival times that both sides consume.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used in counter mode: draw j of
a stream with seed s mixes z = s + (j + 1) * GAMMA (mod 2**64). A draw is
mapped to a double in [0, 1) from its top 53 bits, so every value is exact in
FP64. The paper only says its initial conditions are random (Sec. 3.2); the
uniform law on [-1, 1) and the (q, p) interleaving are the readings used here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_TWO_M53 = 1.0 / float(1 << 53)


def splitmix64(seed: int, idx) -> np.ndarray:
    """SplitMix64 output number ``idx`` (0-based, array-like) of stream ``seed``."""
    j = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (j + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, idx) -> np.ndarray:
    """Doubles in [0, 1) with 53 random bits, from SplitMix64 draws."""
    z = splitmix64(seed, idx)
    return (z >> np.uint64(11)).astype(np.float64) * _TWO_M53


def _chunks(n: int, chunk: int = 1 << 22):
    for a in range(0, n, chunk):
        yield a, min(n, a + chunk)


def chain_ics(n: int, seed: int = 0, dtype=np.float64):
    """Initial (q, p) for an n-site chain, both uniform on [-1, 1).

    q_i uses draw 2i and p_i draw 2i + 1 of stream ``seed``. With
    ``dtype=np.float32`` the FP64 values are rounded to nearest.
    """
    if n < 0:
        raise ValueError("n must be >= 0")
    q = np.empty(n, dtype=np.float64)
    p = np.empty(n, dtype=np.float64)
    for a, b in _chunks(n):
        i = np.arange(a, b, dtype=np.uint64)
        q[a:b] = 2.0 * uniform01(seed, 2 * i) - 1.0
        p[a:b] = 2.0 * uniform01(seed, 2 * i + 1) - 1.0
    if dtype != np.float64:
        q = q.astype(dtype)
        p = p.astype(dtype)
    return q, p


def roessler_ics(n: int, seed: int = 0):
    """Random initial (x, y, z) for an n-site Roessler chain (the paper starts
    from random initial conditions, Sec. 3.2, without saying which): all three
    uniform on [-1, 1), like the other chains. Site i uses draws 3i, 3i + 1,
    3i + 2 of stream ``seed``."""
    if n < 0:
        raise ValueError("n must be >= 0")
    x, y, z = (np.empty(n, dtype=np.float64) for _ in range(3))
    for a, b in _chunks(n):
        i = np.arange(a, b, dtype=np.uint64)
        x[a:b] = 2.0 * uniform01(seed, 3 * i) - 1.0
        y[a:b] = 2.0 * uniform01(seed, 3 * i + 1) - 1.0
        z[a:b] = 2.0 * uniform01(seed, 3 * i + 2) - 1.0
    return x, y, z


def _as_i64(x: int) -> int:
    x &= 0xFFFFFFFFFFFFFFFF
    return x - (1 << 64) if x >= (1 << 63) else x


def chain_ics_torch(n: int, seed: int, device, dtype=None, chunk: int = 1 << 26):
    """Same values as ``chain_ics``, generated with torch on ``device``, in
    chunks of ``chunk`` sites (so very long chains need no large temporaries).

    The 64-bit arithmetic runs in int64 (wrapping multiply; logical shifts by
    masking the sign-extended arithmetic shift).
    """
    import torch

    dtype = dtype or torch.float64

    def lsr(z, k):
        return (z >> k) & ((1 << (64 - k)) - 1)

    def draw(j):
        z = _as_i64(seed) + (j + 1) * _as_i64(0x9E3779B97F4A7C15)
        z = (z ^ lsr(z, 30)) * _as_i64(0xBF58476D1CE4E5B9)
        z = (z ^ lsr(z, 27)) * _as_i64(0x94D049BB133111EB)
        z = z ^ lsr(z, 31)
        return lsr(z, 11).to(torch.float64) * _TWO_M53

    q = torch.empty(n, device=device, dtype=dtype)
    p = torch.empty(n, device=device, dtype=dtype)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        i = torch.arange(a, b, device=device, dtype=torch.int64)
        q[a:b] = (2.0 * draw(2 * i) - 1.0).to(dtype)
        p[a:b] = (2.0 * draw(2 * i + 1) - 1.0).to(dtype)
    return q, p


def mode_ics(n: int, kind: str, amp: float = 0.5, mode: int = 1):
    """Structured initial conditions with closed-form solutions.

    ``uniform``: q_i = amp, p_i = 0.
    ``pi``: q_i = (-1)^i amp, p_i = 0 (n even).
    ``cos``: q_i = amp * cos(2 pi mode i / n), p_i = 0.
    """
    i = np.arange(n, dtype=np.float64)
    if kind == "uniform":
        q = np.full(n, amp)
    elif kind == "pi":
        if n % 2:
            raise ValueError("the pi mode needs an even chain length")
        q = np.where(np.arange(n) % 2 == 0, amp, -amp).astype(np.float64)
    elif kind == "cos":
        q = amp * np.cos(2.0 * math.pi * mode * i / n)
    else:
        raise ValueError(kind)
    return q, np.zeros(n)


# ---------------------------------------------------------------------------
# Batched and served workloads.
# ---------------------------------------------------------------------------

def batch_lengths(count: int, lo: int = 256, hi: int = 65536, seed: int = 4096) -> np.ndarray:
    """Chain lengths log-uniform on [lo, hi]: round(lo * (hi/lo)**u)."""
    u = uniform01(seed, np.arange(count, dtype=np.uint64))
    return np.rint(lo * np.power(hi / lo, u)).astype(np.int64)


@dataclass(frozen=True)
class Job:
    """One integration request of the served workload."""
    jid: int
    arrival: float      # seconds after the start of the run
    n: int              # chain length
    steps: int          # RK4 steps requested
    prec: int           # 0 = FP64, 1 = FP32 with compensated update
    model: int          # 0 = quartic, 1 = harmonic
    seed: int           # initial-condition stream


def served_jobs(count: int, rate: float, seed: int = 5, n_lo: int = 1000,
                n_hi: int = 4_000_000, steps_lo: int = 1000,
                steps_hi: int = 100_000) -> list[Job]:
    """Poisson arrivals with rate ``rate`` per second; per-job draws from
    stream ``seed``: n log-uniform on [n_lo, n_hi], steps uniform integer on
    [steps_lo, steps_hi], precision and model each a fair coin."""
    jobs = []
    t = 0.0
    for j in range(count):
        base = np.arange(6 * j, 6 * j + 6, dtype=np.uint64)
        u = uniform01(seed, base)
        t += -math.log1p(-u[0]) / rate
        n = int(round(n_lo * (n_hi / n_lo) ** u[1]))
        steps = steps_lo + int(math.floor(u[2] * (steps_hi - steps_lo + 1)))
        jobs.append(Job(j, t, n, steps, int(u[3] < 0.5), int(u[4] < 0.5),
                        1_000_000 + j))
    return jobs
