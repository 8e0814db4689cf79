"""CPU FP64 oracle for classical RK4 on a periodic nearest-neighbour chain.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers. Nothing here is shared with the GPU
library. The arithmetic lives in ``chain_oracle.c`` (plain C, FP64, no FMA);
this module only marshals numpy arrays into it.

Model ids: 0 = quartic chain, 1 = harmonic chain, 3 and 4 = the same with
second-neighbour bonds (see ``chain_oracle.c``); the Roessler chain (three
coordinates per site) has its own calls.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "chain_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")
# A test may point the wrapper at another build of the oracle (a copy with a
# planted mistake) to check that the pins catch it.
_LIB_OVERRIDE = os.environ.get("CHAIN_ORACLE_LIB")

QUARTIC = 0
HARMONIC = 1
QUARTIC_NNN = 3
HARMONIC_NNN = 4


def coupling_range(model: int) -> int:
    """Farthest neighbour a site's force reads (1 or 2)."""
    return 2 if model in (QUARTIC_NNN, HARMONIC_NNN) else 1
# The paper's Roessler parameters (Sec. 3.1): a = 0.2, b = 1, c = 9.
ROESSLER_ABC = (0.2, 1.0, 9.0)


def build(force: bool = True, src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle with gcc: -O3 for generic x86-64 (the library file
    also runs on hosts other than the one that built it), no FMA contraction
    and no fast-math, so every operation rounds as written; OpenMP."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               src, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _LIB_OVERRIDE or LIB
        if path == LIB and not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_force.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp]
        lib.oracle_force.restype = None
        lib.oracle_rk4_run.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                       ctypes.c_int64, dp, dp, ctypes.c_int]
        lib.oracle_rk4_run.restype = ctypes.c_int
        lib.oracle_energy.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp]
        lib.oracle_rk_tableau_run.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                              ctypes.c_int64, dp, dp, ctypes.c_int, dp, dp,
                                              ctypes.c_int]
        lib.oracle_rk_tableau_run.restype = ctypes.c_int
        lib.oracle_energy.restype = ctypes.c_double
        d = ctypes.c_double
        lib.oracle_roessler_rhs.argtypes = [ctypes.c_int64, dp, dp, dp, d, d, d, dp, dp, dp]
        lib.oracle_roessler_rhs.restype = None
        lib.oracle_roessler_run.argtypes = [ctypes.c_int64, d, ctypes.c_int64, dp, dp, dp, d, d, d,
                                            ctypes.c_int]
        lib.oracle_roessler_run.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def force(model: int, q) -> np.ndarray:
    """F(q) for every site of the ring."""
    q = _f64(q)
    f = np.empty_like(q)
    _load().oracle_force(model, q.size, _ptr(q), _ptr(f))
    return f


def rk4(model: int, q, p, dt: float, steps: int, threads: int = 1):
    """Return (q, p) after ``steps`` RK4 steps of size ``dt`` (copies)."""
    q = _f64(q).copy()
    p = _f64(p).copy()
    if q.shape != p.shape or q.ndim != 1:
        raise ValueError("q and p must be 1-D arrays of one length")
    rc = _load().oracle_rk4_run(model, q.size, float(dt), int(steps), _ptr(q), _ptr(p),
                                int(threads))
    if rc != 0:
        raise MemoryError("oracle_rk4_run failed")
    return q, p


def rk_tableau(model: int, q, p, dt: float, steps: int, a, b, threads: int = 1):
    """(q, p) after ``steps`` steps of the explicit Runge-Kutta method with
    coefficients ``a`` (s x s, strictly lower triangle used) and weights ``b``."""
    q = _f64(q).copy()
    p = _f64(p).copy()
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    s = b.size
    if a.shape != (s, s) or q.shape != p.shape or q.ndim != 1:
        raise ValueError("a must be s x s for s weights; q and p 1-D of one length")
    rc = _load().oracle_rk_tableau_run(model, q.size, float(dt), int(steps), _ptr(q), _ptr(p),
                                       int(s), _ptr(a), _ptr(b), int(threads))
    if rc != 0:
        raise MemoryError("oracle_rk_tableau_run failed")
    return q, p


def energy(model: int, q, p) -> float:
    """Total energy of the ring (compensated sum in index order)."""
    q = _f64(q)
    p = _f64(p)
    return float(_load().oracle_energy(model, q.size, _ptr(q), _ptr(p)))


def rk4_sites(model: int, q, p, dt: float, steps: int, sites, threads: int = 1):
    """Final (q, p) of selected sites only, each from its own light cone.

    After ``steps`` RK4 steps a site depends on the initial state within
    4 * range * steps sites of it (``range`` sites per stage, Sec. 2.3 and
    Sec. 5). On a ring of 2 * 4 * range * steps + 1 sites cut from the chain
    around site i, those sites are the same, so site i comes out exactly as on
    the full ring. Used when the full ring is too long for the oracle; chains
    shorter than the window run whole.
    """
    q = _f64(q)
    p = _f64(p)
    n = q.size
    r = 4 * coupling_range(model) * int(steps)
    w = 2 * r + 1
    sites = np.asarray(sites, dtype=np.int64)
    if w >= n:
        qf, pf = rk4(model, q, p, dt, steps, threads)
        return qf[sites], pf[sites]
    oq = np.empty(sites.size)
    op = np.empty(sites.size)
    for k, i in enumerate(sites):
        idx = (np.arange(i - r, i + r + 1) % n)
        qw, pw = rk4(model, q[idx], p[idx], dt, steps, threads)
        oq[k] = qw[r]
        op[k] = pw[r]
    return oq, op


def roessler_rhs(x, y, z, abc=ROESSLER_ABC):
    """(dx/dt, dy/dt, dz/dt) of the Roessler chain."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    kx, ky, kz = np.empty_like(x), np.empty_like(x), np.empty_like(x)
    _load().oracle_roessler_rhs(x.size, _ptr(x), _ptr(y), _ptr(z), *abc, _ptr(kx), _ptr(ky), _ptr(kz))
    return kx, ky, kz


def roessler_rk4(x, y, z, dt: float, steps: int, abc=ROESSLER_ABC, threads: int = 1):
    """Return (x, y, z) after ``steps`` RK4 steps of the Roessler chain."""
    x, y, z = _f64(x).copy(), _f64(y).copy(), _f64(z).copy()
    if not (x.shape == y.shape == z.shape) or x.ndim != 1:
        raise ValueError("x, y, z must be 1-D arrays of one length")
    rc = _load().oracle_roessler_run(x.size, float(dt), int(steps), _ptr(x), _ptr(y), _ptr(z),
                                     *abc, int(threads))
    if rc != 0:
        raise MemoryError("oracle_roessler_run failed")
    return x, y, z


def roessler_rk4_sites(x, y, z, dt: float, steps: int, sites, abc=ROESSLER_ABC, threads: int = 1):
    """Final (x, y, z) of selected sites, each from its own light cone of
    2 * 4 * steps + 1 sites (see rk4_sites)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    r = 4 * int(steps)
    sites = np.asarray(sites, dtype=np.int64)
    if 2 * r + 1 >= n:
        a, b, c = roessler_rk4(x, y, z, dt, steps, abc, threads)
        return a[sites], b[sites], c[sites]
    out = np.empty((3, sites.size))
    for k, i in enumerate(sites):
        idx = np.arange(i - r, i + r + 1) % n
        a, b, c = roessler_rk4(x[idx], y[idx], z[idx], dt, steps, abc, threads)
        out[:, k] = a[r], b[r], c[r]
    return out[0], out[1], out[2]
