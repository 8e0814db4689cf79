"""The hand-off of the register-resident Roessler run (CHAIN_FLAG_EXCHANGE),
emulated on the CPU with the library's own plans: clusters keep balanced
tiles, write the kept sites their neighbours read after each pass, mark the
pass done, wait for both neighbours and reload their halo; exchange buffers
alternate by pass parity and the last (odd) pass stores into the caller's
buffers. Clusters advance in random interleavings that respect only those
waits. Each value is a tag (site, passes applied) instead of a number, so the
emulation checks that every access is inside the arrays, that every halo
site a cluster reads is its neighbour's value of the same pass (never an
older or a newer one), and that the caller's buffers end with every site
advanced by every pass."""
import ctypes
import random

import pytest

from paper_1412_0544_amd import _lib as L

REACH = 4   # sites one Roessler step carries a change (pinned on the oracle)


def plan_for(n, sites, waves, depth):
    d = L.Desc(n, L.CHAIN_ROESSLER, L.CHAIN_FP64, 0.01, L.CHAIN_FUSED, sites, depth, waves,
               L.CHAIN_FLAG_EXCHANGE, 0)
    P = L.Plan()
    rc = L.lib().chain_rk4_plan_for(ctypes.byref(d), None, ctypes.byref(P))
    return rc, P


def layout(n, P):
    """(G, uq, ur, halo, zone) the way the library plans them."""
    E = 64 * P.sites_per_lane * P.waves_per_cluster
    tmax = E - 2 * P.halo
    G = -(-n // (tmax - 4))
    uq, ur = (n // 4) // G, (n // 4) % G
    return E, G, uq, ur, P.halo, E - P.halo - 4 * uq


def emulate(n, P, steps, rng, flags=None, fbase=0, front=None):
    """One step call. `flags` (per cluster) carry over from the previous
    call, all at `fbase`; `front` holds (site, passes) tags. Returns the
    cluster count and the pass count."""
    E, G, uq, ur, halo, zone = layout(n, P)
    assert (G, 4 * (uq + 1), zone) == (P.waves, P.tile, zone)
    passes = -(-steps // P.kdepth)
    passes += passes % 2
    base, extra = divmod(steps, passes)
    assert all(base + (j < extra) <= P.kdepth for j in range(passes))
    assert halo >= REACH * P.kdepth
    if front is None:
        front = [(i, 0) for i in range(n)]      # the caller's buffers: tags (site, passes)
    p0 = front[0][1]
    back = [None] * n
    if flags is None:
        flags = [0] * G

    def cluster(g):
        start = 4 * (g * uq + min(g, ur))
        keep = n - start if g == G - 1 else 4 * (uq + (1 if g < ur else 0))
        e0 = start - halo
        left, right = (g - 1) % G, (g + 1) % G
        # load: the window, wrapped (any sign; the kernel wraps by index)
        win = [(site, p - p0) for site, p in (front[(e0 + loc) % n] for loc in range(E))]
        assert all(t[1] == 0 for t in win)
        for j in range(passes):
            yield ("compute", g, j)
            # a site is exact after the pass iff its local position is at
            # least reach*k from both window ends: the kept ones are
            k = base + (1 if j < extra else 0)
            for loc in range(E):
                site, p = win[loc]
                assert site == (e0 + loc) % n
                exact = REACH * k <= loc < E - REACH * k
                win[loc] = (site, p + 1) if exact and p == j else (site, None)
            for loc in range(halo, halo + keep):
                assert win[loc] == ((e0 + loc) % n, j + 1), (g, j, loc)
            if j + 1 == passes:
                break
            ex = front if j % 2 else back
            for loc in range(halo, halo + keep):
                if loc < halo + zone or loc >= keep:
                    site = e0 + loc
                    assert 0 <= site < n            # kept sites never wrap
                    ex[site] = win[loc]
            flags[g] = fbase + j + 1
            while not (flags[left] >= fbase + j + 1 and flags[right] >= fbase + j + 1):
                yield ("wait", g, j)
            for loc in range(E):
                if loc < halo or loc >= halo + keep:
                    i = e0 + loc
                    i = i + n if i < 0 else (i - n if i >= n else i)
                    assert 0 <= i < n
                    win[loc] = ex[i]
                    assert win[loc] == (i, j + 1), (g, j, loc, win[loc])
        for loc in range(halo, halo + keep):
            site, p = win[loc]
            front[e0 + loc] = (site, p + p0)
        yield ("done", g, passes)

    runners = {g: cluster(g) for g in range(G)}
    while runners:
        g = rng.choice(list(runners))
        try:
            next(runners[g])
        except StopIteration:
            del runners[g]
    assert front == [(i, p0 + passes) for i in range(n)]
    # every cluster sets its counter after each pass but the last
    assert flags == [fbase + passes - 1] * G
    return G, passes


@pytest.mark.parametrize("sites,waves,depth,n,steps", [
    (4, 4, 25, 20011, 50), (4, 4, 13, 9000, 50), (4, 1, 6, 4001, 37), (8, 2, 20, 30011, 61),
    (4, 2, 1, 2051, 2), (4, 4, 16, 8195, 1000), (8, 1, 11, 6007, 23), (4, 8, 32, 40003, 64),
    (4, 4, 25, 2000, 50),
])
def test_exchange_hand_off_in_random_orders(sites, waves, depth, n, steps):
    rc, P = plan_for(n, sites, waves, depth)
    assert rc == L.CHAIN_OK and P.exchange == 1
    for seed in range(3):
        G, passes = emulate(n, P, steps, random.Random(seed))
        assert G >= 3 and passes % 2 == 0


@pytest.mark.parametrize("sites,waves,depth,n", [(4, 4, 25, 20011), (4, 2, 7, 5003)])
def test_progress_counters_carry_over_successive_calls(sites, waves, depth, n):
    """The counters are not cleared between calls: a call starts from the
    value they all hold after the previous one (base + passes - 1)."""
    rc, P = plan_for(n, sites, waves, depth)
    assert rc == L.CHAIN_OK and P.exchange == 1
    rng = random.Random(5)
    G = P.waves
    flags, fbase, front = [0] * G, 0, [(i, 0) for i in range(n)]
    for steps in (50, 2, 3 * depth + 1, 7, 50):
        _, passes = emulate(n, P, steps, rng, flags, fbase, front)
        fbase += passes - 1


def test_a_stale_base_lets_a_cluster_read_an_old_halo():
    """Planted mistake, on the CPU: a call that starts below the counters'
    value (as a replayed graph would, had it not cleared them) lets some
    cluster pass its wait before its neighbours' edges are written."""
    n, sites, waves, depth = 20011, 4, 4, 25
    rc, P = plan_for(n, sites, waves, depth)
    assert rc == L.CHAIN_OK
    caught = 0
    for seed in range(6):
        flags = [0] * P.waves
        front = [(i, 0) for i in range(n)]
        emulate(n, P, 50, random.Random(seed), flags, 0, front)
        try:
            emulate(n, P, 50, random.Random(100 + seed), flags, 0, front)  # stale base 0
        except AssertionError:
            caught += 1
    assert caught > 0


def test_exchange_plans_refused_when_clusters_cannot_hand_off():
    # too short for three clusters, and a chain no longer than one cluster
    for n in (100, 1024, 1500):
        rc, _ = plan_for(n, 4, 4, 25)
        assert rc == L.CHAIN_EINVAL
    d = L.Desc(1 << 20, L.CHAIN_QUARTIC, 0, 0.01, 0, 0, 0, 0, L.CHAIN_FLAG_EXCHANGE, 0)
    assert L.lib().chain_rk4_plan_for(ctypes.byref(d), None, ctypes.byref(L.Plan())) == \
        L.CHAIN_EINVAL                                    # the Roessler chain only
    # the paper's workload: N = 2^20 at the default shape
    rc, P = plan_for(1 << 20, 0, 0, 0)
    assert rc == L.CHAIN_OK and P.exchange == 1 and P.waves >= 3
