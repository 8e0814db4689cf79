"""Every plan the library accepts puts each cluster on a 16-byte boundary.

A lane loads and stores its S consecutive sites with 16-byte vector accesses
(two FP64 or four FP32 values) whenever its cluster does not wrap around the
ring, so every cluster origin cluster * tile - halo must be a whole number of
such vectors. The planners round the halo up to one; a wider overlap than a
step's reach keeps the kept sites exact (Sec. 2.3), so this changes no bit of
the result. No GPU is needed: the planners are plain host code.
"""
import ctypes
import os
import sys

import numpy as np
import pytest

from paper_1412_0544_amd import _lib as L
from paper_1412_0544_amd.chain import make_tableau

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_oracle_tableau import TABLEAUS, step_reach  # noqa: E402

MODELS = (L.CHAIN_QUARTIC, L.CHAIN_HARMONIC, L.CHAIN_ROESSLER, L.CHAIN_QUARTIC_NNN,
          L.CHAIN_HARMONIC_NNN)
PRECS = (L.CHAIN_FP64, L.CHAIN_FP32_KAHAN, L.CHAIN_FP32_KAHAN64, L.CHAIN_FP32)
# lengths on both sides of every row of the library's shape table
LENGTHS = (1, 2, 100, 4097, (1 << 17), (1 << 17) + 1, (1 << 19) + 1, (1 << 21) + 1,
           (1 << 23) + 1, 1 << 24)


def vector_sites(prec):
    return 2 if prec == L.CHAIN_FP64 else 4


def step_reach_of(model):
    """Sites one step of classical RK4 carries a change (pinned on the oracle:
    test_oracle_tableau's and test_oracle_nnn's exact-reach pins)."""
    return {L.CHAIN_QUARTIC: 2, L.CHAIN_HARMONIC: 2, L.CHAIN_QUARTIC_NNN: 4,
            L.CHAIN_HARMONIC_NNN: 4, L.CHAIN_ROESSLER: 4}[model]


def plan(n, model, prec, s, w, k, flags=0, tab=None):
    scheme = L.CHAIN_SCHEME_RK4 if tab is None else L.CHAIN_SCHEME_TABLEAU
    d = L.Desc(n, model, prec, 0.01, L.CHAIN_FUSED, s, k, w, flags, scheme)
    P = L.Plan()
    t = None if tab is None else ctypes.byref(tab)
    rc = L.lib().chain_rk4_plan_for(ctypes.byref(d), t, ctypes.byref(P))
    return rc, P


def check_aligned(P, prec, reach, where):
    V = vector_sites(prec)
    E = 64 * P.sites_per_lane * P.waves_per_cluster
    assert P.halo % V == 0 and P.tile % V == 0, where
    assert P.halo >= reach * P.kdepth and P.halo < reach * P.kdepth + V, where
    assert P.tile >= 1 and P.tile + 2 * P.halo == E, where
    for c in (0, 1, 2, P.waves - 1):                      # cluster origins
        assert (c * P.tile - P.halo) % V == 0, where


def test_every_classical_plan_is_aligned():
    checked = 0
    for model in MODELS:
        for prec in PRECS:
            for n in LENGTHS:
                for s in (0, 2, 4, 6, 8, 16):      # 6: the Roessler chain only
                    for w in (0, 1, 2, 4, 8):
                        for k in range(0, 33):
                            rc, P = plan(n, model, prec, s, w, k)
                            if rc != L.CHAIN_OK:
                                assert rc == L.CHAIN_EINVAL
                                continue
                            assert P.resident == 0
                            check_aligned(P, prec, step_reach_of(model),
                                          (n, model, prec, s, w, k))
                            if k:
                                assert P.kdepth <= k
                            checked += 1
    # FP64 and the three FP32 forms of four models, and FP64 Roessler chains
    assert checked > 20000


def test_plans_that_used_to_be_misaligned():
    """Odd depths with FP32 state (halo 2 mod 4) and the default plan of a
    tableau with an odd reach (Dormand-Prince 5: reach 3, depth 21)."""
    rc, P = plan(1 << 20, L.CHAIN_QUARTIC, L.CHAIN_FP32_KAHAN, 8, 4, 7)
    assert rc == L.CHAIN_OK and P.halo == 16 and P.kdepth == 7
    rc, P = plan(1 << 20, L.CHAIN_QUARTIC, L.CHAIN_FP64, 8, 4, 7)
    assert rc == L.CHAIN_OK and P.halo == 14
    (a, b), _ = TABLEAUS["dopri5"]
    rc, P = plan(1 << 24, L.CHAIN_QUARTIC, L.CHAIN_FP64, 0, 0, 0,
                 tab=make_tableau(a.tolist(), b.tolist()))
    assert rc == L.CHAIN_OK and P.kdepth == 21 and P.halo == 64 and P.tile == 896


def random_tableaus(seed=7, count=24):
    """Explicit tableaus of 1..8 stages with random zero patterns, so that the
    reach per step takes many values (odd ones included)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        s = 1 + i % 8
        a = np.tril(rng.uniform(-1, 1, (s, s)), -1)
        a[rng.uniform(size=(s, s)) < 0.4] = 0.0
        b = rng.uniform(0.1, 1.0, s)
        b[rng.uniform(size=s) < 0.3] = 0.0
        if not b.any():
            b[-1] = 1.0
        out.append((a, b))
    return out


def test_every_tableau_plan_is_aligned():
    tabs = [ab for ab, _ in TABLEAUS.values()] + random_tableaus()
    checked = 0
    for a, b in tabs:
        t = make_tableau(a.tolist(), b.tolist())
        for model, rng_ in ((L.CHAIN_QUARTIC, 1), (L.CHAIN_HARMONIC, 1),
                            (L.CHAIN_QUARTIC_NNN, 2), (L.CHAIN_HARMONIC_NNN, 2)):
            reach = max(1, step_reach(np.asarray(a), np.asarray(b), rng_))
            for prec in (L.CHAIN_FP64, L.CHAIN_FP32_KAHAN):
                for n in (5003, 1 << 24):
                    for s in (0, 4, 8):
                        for w in (0, 1, 4):
                            for k in range(0, 33):
                                rc, P = plan(n, model, prec, s, w, k, tab=t)
                                if rc != L.CHAIN_OK:
                                    assert rc == L.CHAIN_EINVAL
                                    continue
                                check_aligned(P, prec, reach, (len(b), model, prec, s, w, k))
                                checked += 1
    assert checked > 5000


@pytest.mark.parametrize("flags", [0, L.CHAIN_BATCH_FENCES])
def test_every_batch_shape_is_aligned(flags):
    from paper_1412_0544_amd.batch import Batch
    for s in (0, 4, 8, 16):
        for k in [0] + list(range(2, 33)):
            P = Batch.plan_for(s, k, flags)
            E = 64 * P["sites_per_lane"] * P["waves_per_cluster"]
            halo, depth = P["halo"], P["kdepth"]
            # tiles start at multiples of 4 sites; the origin start - halo too
            assert halo % 4 == 0 and 2 * depth <= halo < 2 * depth + 4, (s, k)
            assert P["tile_max"] + 2 * halo == E and P["tile_max"] % 4 == 0
            # a cluster keeps at least `halo` sites whenever a chain has two
            # or more, so it reads only its own and its neighbours' tiles
            assert E >= 4 * halo + 16, (s, k)


def test_plan_for_validates_like_create():
    lib = L.lib()
    P = L.Plan()
    d = L.Desc(1000, 0, 0, 0.01, 0, 0, 0, 0, 0, 0)
    assert lib.chain_rk4_plan_for(ctypes.byref(d), None, None) == L.CHAIN_EINVAL
    assert lib.chain_rk4_plan_for(None, None, ctypes.byref(P)) == L.CHAIN_EINVAL
    (a, b), _ = TABLEAUS["rk4"]
    t = make_tableau(a.tolist(), b.tolist())
    # a tableau only with the tableau scheme, and always with it
    assert lib.chain_rk4_plan_for(ctypes.byref(d), ctypes.byref(t), ctypes.byref(P)) == L.CHAIN_EINVAL
    d.scheme = L.CHAIN_SCHEME_TABLEAU
    assert lib.chain_rk4_plan_for(ctypes.byref(d), None, ctypes.byref(P)) == L.CHAIN_EINVAL
    assert lib.chain_rk4_plan_for(ctypes.byref(d), ctypes.byref(t), ctypes.byref(P)) == L.CHAIN_OK
    assert P.halo == 64 and P.kdepth == 32
    d.sites_per_lane = 2                          # the tableau kernel takes S = 4 or 8
    assert lib.chain_rk4_plan_for(ctypes.byref(d), ctypes.byref(t), ctypes.byref(P)) == L.CHAIN_EINVAL
    bd = L.BatchDesc(10, 0, 5, 0, 0, 0, 0, 0)
    assert lib.chain_rk4_batch_plan_for(ctypes.byref(bd), ctypes.byref(L.BatchPlan())) == L.CHAIN_EINVAL
    # the headline plan: N = 2^24 FP64, S=8 W=4 k=32, halo 64, tile 1920
    rc, P = plan(1 << 24, L.CHAIN_QUARTIC, L.CHAIN_FP64, 0, 0, 0)
    assert rc == L.CHAIN_OK and (P.sites_per_lane, P.waves_per_cluster, P.kdepth) == (8, 4, 32)
    assert (P.halo, P.tile, P.waves) == (64, 1920, -(-(1 << 24) // 1920))
    # chains that fill the chip about once: 6 sites per lane at 2^18-2^19 and
    # in four-wavefront clusters at 2^21
    for n, shape in ((1 << 10, (2, 1, 28)), (1 << 14, (2, 1, 28)), ((1 << 14) + 1, (2, 1, 16)),
                     (1 << 16, (2, 1, 16)), (1 << 17, (4, 1, 32)), (1 << 19, (6, 1, 32)),
                     (1 << 20, (8, 1, 32)), (1 << 21, (6, 4, 32)), ((1 << 21) + 1, (8, 4, 32))):
        rc, P = plan(n, L.CHAIN_QUARTIC, L.CHAIN_FP64, 0, 0, 0)
        assert rc == L.CHAIN_OK
        assert (P.sites_per_lane, P.waves_per_cluster, P.kdepth) == shape, n
    # the Roessler chain (fused passes) and the FP64 second-neighbour chains
    for model, rows in ((L.CHAIN_ROESSLER, ((1 << 10, (4, 1, 25)), (1 << 16, (4, 1, 16)),
                                            (1 << 18, (8, 1, 25)), (1 << 20, (4, 4, 25)),
                                            (1 << 24, (8, 4, 25)))),
                        (L.CHAIN_QUARTIC_NNN, ((1 << 10, (2, 1, 14)), (1 << 16, (2, 1, 8)),
                                               (1 << 18, (4, 1, 16)), (1 << 20, (8, 1, 16)),
                                               (1 << 24, (8, 4, 16))))):
        for n, shape in rows:
            rc, P = plan(n, model, L.CHAIN_FP64, 0, 0, 0)
            assert rc == L.CHAIN_OK
            assert (P.sites_per_lane, P.waves_per_cluster, P.kdepth) == shape, (model, n)
    # the FP32 forms of the second-neighbour chains
    for prec in (L.CHAIN_FP32_KAHAN, L.CHAIN_FP32):
        for n, shape in ((1 << 10, (2, 1, 14)), (1 << 16, (2, 1, 8)), (1 << 18, (4, 1, 16)),
                         (1 << 20, (4, 4, 16)), (1 << 22, (8, 4, 16)), (1 << 24, (16, 4, 16))):
            rc, P = plan(n, L.CHAIN_HARMONIC_NNN, prec, 0, 0, 0)
            assert rc == L.CHAIN_OK
            assert (P.sites_per_lane, P.waves_per_cluster, P.kdepth) == shape, (prec, n)
    # tableau passes: one wavefront of 4 sites per lane up to 2^18 sites, then
    # four wavefronts (of 4 sites per lane up to 2^20 for compensated FP32)
    for name, depth, long_sites in (("rk4_38", 32, 8), ("dopri5", 21, 4)):
        (a, b), _ = TABLEAUS[name]
        t = make_tableau(a.tolist(), b.tolist())
        for prec, mid in ((L.CHAIN_FP64, long_sites), (L.CHAIN_FP32_KAHAN, 4)):
            for n, shape in ((1 << 10, (4, 1, depth)), (1 << 18, (4, 1, depth)),
                             ((1 << 18) + 1, (mid, 4, depth)),
                             ((1 << 20) + 1, (long_sites, 4, depth))):
                if name == "rk4_38" and prec == L.CHAIN_FP64 and n == (1 << 18) + 1:
                    shape = (8, 1, depth)      # four stages: one wavefront up to 2^20
                rc, P = plan(n, L.CHAIN_QUARTIC, prec, 0, 0, 0, tab=t)
                assert rc == L.CHAIN_OK
                assert (P.sites_per_lane, P.waves_per_cluster, P.kdepth) == shape, (name, prec, n)
    # the FP32 forms: the same short-chain rows, then four-wavefront clusters
    for prec in (L.CHAIN_FP32_KAHAN, L.CHAIN_FP32):
        for n, shape in ((1 << 10, (2, 1, 28)), (1 << 14, (2, 1, 28)), (1 << 16, (2, 1, 16)),
                         (1 << 17, (4, 1, 32)), (1 << 18, (2, 4, 32))):
            rc, P = plan(n, L.CHAIN_QUARTIC, prec, 0, 0, 0)
            assert rc == L.CHAIN_OK
            assert (P.sites_per_lane, P.waves_per_cluster, P.kdepth) == shape, (prec, n)
