"""How the batch cuts a chain into clusters, checked on the CPU.

A tiled chain is cut into wide clusters (four wavefronts, 64*S*4 sites)
followed by at most three narrow ones (one wavefront, 64*S sites). Every
cluster pass recomputes `halo` sites on each side and keeps the rest (the
overlap of Sec. 2.3), so any cut whose kept ranges tile the ring gives the
same result; the cut only decides how many lane-sites a pass occupies. These
tests pin the rules the kernel relies on (aligned starts, kept ranges that
tile [0, n), every cluster of a multi-cluster chain keeping at least `halo`
sites so its neighbours' halos lie in the adjacent clusters) and that the
cut is the cheapest one, against a brute-force search written here.
"""
import numpy as np
import pytest

from paper_1412_0544_amd import _lib as L
from paper_1412_0544_amd.batch import Batch

SHAPES = [(4, 32), (8, 32), (8, 12), (16, 32), (4, 8), (8, 2), (16, 5)]
LENGTHS = sorted(set([1, 2, 3, 4, 5, 7, 63, 64, 100, 255, 256, 257, 383, 384, 385, 500, 511, 512,
                      767, 1000, 1023, 1024, 1025, 1500, 1900, 1919, 1920, 1921, 2047, 2048, 2300,
                      3000, 3839, 3840, 4000, 5003, 7777, 20011, 65536, 100_000, 1 << 20])
                 | set(int(x) for x in np.random.default_rng(7).integers(1, 70_000, 60)))


def cheapest(n, P):
    """Fewest lane-sites over every (wide, narrow) count that can hold n:
    brute force over the counts, each cluster holding at most tile - 4
    sites in whole units of 4 (the last one the n % 4 remainder too) and, with
    two or more clusters, at least halo sites."""
    S, halo = P["sites_per_lane"], P["halo"]
    E4, E1 = 64 * S * 4, 64 * S
    t4, t1 = P["tile_max"], P["tile_narrow"]
    best = None
    for g1 in range(0, (8 if t1 else 0) + 1):
        for g4 in range(0, n // max(t4 - 4, 1) + 3):
            G = g4 + g1
            if G == 0:
                continue
            units = n // 4
            cap = g4 * (t4 // 4 - 1) + g1 * ((t1 // 4 - 1) if t1 else 0)
            if units > cap or (G >= 2 and units < G * (halo // 4)):
                continue
            cost = g4 * E4 + g1 * E1
            if best is None or cost < best:
                best = cost
    return best


@pytest.mark.parametrize("S,K", SHAPES)
@pytest.mark.parametrize("flags", [0, L.CHAIN_BATCH_WIDE_ONLY])
def test_cut_tiles_the_ring_and_is_the_cheapest(S, K, flags):
    P = Batch.plan_for(S, K, flags)
    halo, E4, E1 = P["halo"], 64 * S * 4, 64 * S
    if flags or E1 < 4 * halo + 16:
        assert P["tile_narrow"] == 0
    else:
        assert P["tile_narrow"] == E1 - 2 * halo
    for n in LENGTHS:
        cut = Batch.layout(n, S, K, flags)
        starts = [c[0] for c in cut]
        keeps = [c[1] for c in cut]
        waves = [c[2] for c in cut]
        # kept ranges tile [0, n) in order, starting on 16-byte boundaries
        assert starts[0] == 0 and sum(keeps) == n
        assert all(a + k == b for a, k, b in zip(starts, keeps, starts[1:]))
        assert all(a % 4 == 0 and (a - halo) % 4 == 0 for a in starts)
        # wide clusters first, at most three narrow ones after them
        nw = waves.count(4)
        assert waves == [4] * nw + [1] * (len(cut) - nw) and len(cut) - nw <= 3
        if P["tile_narrow"] == 0:
            assert nw == len(cut)
        for k, w in zip(keeps, waves):
            assert 0 < k < (P["tile_max"] if w == 4 else P["tile_narrow"]), (n, cut)
            if len(cut) >= 2:
                assert k >= halo, (n, cut)
        cost = nw * E4 + (len(cut) - nw) * E1
        assert cost == cheapest(n, P), (n, S, K, flags, cut)


def test_mixed_cut_saves_lane_sites_on_the_batch_lengths():
    """On the 4096-chain length mix (log-uniform in [256, 65536]) at 8 sites
    per lane and depth 32, the narrow clusters cut the occupied lane-sites by
    about 5% (kept fraction 0.865 -> 0.909)."""
    import workloads
    lengths = workloads.batch_lengths(4096)
    occ = {}
    for flags in (0, L.CHAIN_BATCH_WIDE_ONLY):
        occ[flags] = sum(sum(64 * 8 * w for _, _, w in Batch.layout(int(n), 8, 32, flags))
                         for n in lengths)
    kept_mixed = lengths.sum() / occ[0]
    kept_wide = lengths.sum() / occ[L.CHAIN_BATCH_WIDE_ONLY]
    assert kept_wide < 0.87 and kept_mixed > 0.905, (kept_wide, kept_mixed)


def test_layout_rejects_bad_arguments():
    import ctypes
    lib = L.lib()
    d = L.BatchDesc(0, 0, 8, 32, 0, 0, 0, 0)
    assert lib.chain_rk4_batch_layout(0, ctypes.byref(d), None, None, None, 0) == -1
    assert lib.chain_rk4_batch_layout(10, None, None, None, None, 0) == -1
    assert lib.chain_rk4_batch_layout(10, ctypes.byref(d), None, None, None, 4) == -1
    bad = L.BatchDesc(0, 0, 5, 32, 0, 0, 0, 0)
    assert lib.chain_rk4_batch_layout(10, ctypes.byref(bad), None, None, None, 0) == -1
    # a short capacity fills only what fits and still returns the count
    start = (ctypes.c_int64 * 1)()
    keep = (ctypes.c_int64 * 1)()
    waves = (ctypes.c_int32 * 1)()
    count = lib.chain_rk4_batch_layout(100_000, ctypes.byref(d), start, keep, waves, 1)
    assert count == len(Batch.layout(100_000, 8, 32)) > 1
    assert start[0] == 0 and waves[0] == 4
