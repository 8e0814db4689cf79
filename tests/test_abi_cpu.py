"""The C-ABI library without a GPU: it loads, exports every declared symbol,
and rejects invalid arguments before touching the HIP runtime."""
import ctypes
import os
import re

import pytest

from paper_1412_0544_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chain_rk4.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chain_rk4_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 10
    lib = L.lib()
    for name in names:
        assert hasattr(lib, name), name


def desc(**kw):
    d = dict(n=1000, model=0, prec=0, dt=0.01, method=0, sites_per_lane=0, kdepth=0,
             waves_per_cluster=0, flags=0, scheme=0)
    d.update(kw)
    return L.Desc(**d)


def test_workspace_bytes():
    lib = L.lib()
    f = lambda d: lib.chain_rk4_workspace_bytes(ctypes.byref(d))
    fused = f(desc(n=1 << 20))
    assert fused >= 2 * 8 * (1 << 20)
    assert f(desc(n=1 << 20, prec=1)) >= 6 * 4 * (1 << 20)
    # per-stage method: stage argument (two arrays), F1, F2 and the force sum
    assert f(desc(n=1 << 20, method=1)) >= 5 * 8 * (1 << 20)
    assert f(desc(n=4096, flags=4)) > 0                            # resident ring
    # per-stage tableau method: 7 force arrays and two stage arguments
    assert f(desc(n=1 << 20, method=1, scheme=1)) >= 9 * 8 * (1 << 20)
    for bad in (desc(n=0), desc(model=7), desc(prec=4), desc(prec=-1), desc(dt=float("nan")),
                desc(dt=float("inf")), desc(method=5), desc(sites_per_lane=5),
                desc(kdepth=33), desc(kdepth=-1), desc(sites_per_lane=2, model=2), desc(sites_per_lane=1), desc(model=5), desc(model=2, prec=1), desc(flags=64), desc(waves_per_cluster=3),
                desc(waves_per_cluster=16), desc(scheme=7), desc(scheme=1, model=2),
                desc(flags=4, n=4097), desc(flags=6), desc(flags=4, model=3),
                desc(flags=4, scheme=1), desc(flags=4, method=1)):
        assert f(bad) == 0
    assert lib.chain_rk4_workspace_bytes(None) == 0


def test_fp64_carry_precision_validation_and_workspace():
    """CHAIN_FP32_KAHAN64 keeps two FP64 carries per site (front and back on
    the fused path): 16 more bytes per site than CHAIN_FP32_KAHAN; resident
    rings, tableaus, the Roessler chain and batches refuse it."""
    lib = L.lib()
    f = lambda d: lib.chain_rk4_workspace_bytes(ctypes.byref(d))
    n = 1 << 20
    assert f(desc(n=n, prec=2)) - f(desc(n=n, prec=1)) == 4 * 4 * n
    assert f(desc(n=n, prec=2, method=1)) - f(desc(n=n, prec=1, method=1)) == 2 * 4 * n
    for m in (0, 1, 3, 4):
        assert f(desc(prec=2, model=m)) > 0
    for bad in (desc(prec=2, flags=4), desc(prec=2, scheme=1), desc(prec=2, model=2)):
        assert f(bad) == 0


def test_plain_fp32_control_precision_validation_and_workspace():
    """CHAIN_FP32 (no compensation) keeps no carries: the workspace of the
    fused path is the FP32 back buffer, 8 bytes per site, below the
    compensated form's 24; the same restrictions as the FP64-carry form."""
    lib = L.lib()
    f = lambda d: lib.chain_rk4_workspace_bytes(ctypes.byref(d))
    n = 1 << 20
    assert f(desc(n=n, prec=1)) - f(desc(n=n, prec=3)) == 4 * 4 * n
    assert f(desc(n=n, prec=0)) - f(desc(n=n, prec=3)) == 2 * 4 * n
    for m in (0, 1, 3, 4):
        assert f(desc(prec=3, model=m)) > 0 and f(desc(prec=3, model=m, method=1)) > 0
    for bad in (desc(prec=3, flags=4), desc(prec=3, scheme=1), desc(prec=3, model=2)):
        assert f(bad) == 0


def test_create_rejects_bad_arguments_before_any_hip_call():
    lib = L.lib()
    h = L.H()
    d = desc()
    ws = lib.chain_rk4_workspace_bytes(ctypes.byref(d))
    fake = 1 << 20  # never dereferenced: validation fails first
    cases = [
        (ctypes.byref(desc(n=0)), fake, fake, fake, ws, L.CHAIN_EINVAL),
        (ctypes.byref(d), None, fake, fake, ws, L.CHAIN_EINVAL),
        (ctypes.byref(d), fake, None, fake, ws, L.CHAIN_EINVAL),
        (ctypes.byref(d), fake + 8, fake, fake, ws, L.CHAIN_EINVAL),
        (ctypes.byref(d), fake, fake, fake, ws - 1, L.CHAIN_ENOMEM),
        (ctypes.byref(d), fake, fake, None, ws, L.CHAIN_EINVAL),
        (ctypes.byref(d), fake, fake, fake + 16, ws, L.CHAIN_EINVAL),
    ]
    for dp, q, p, w, nb, want in cases:
        assert lib.chain_rk4_create(dp, q, p, w, nb, None, ctypes.byref(h)) == want
        assert lib.chain_rk4_last_error()
    assert lib.chain_rk4_create(ctypes.byref(d), fake, fake, fake, ws, None, None) == L.CHAIN_EINVAL


def test_null_handles():
    lib = L.lib()
    assert lib.chain_rk4_destroy(None) == L.CHAIN_OK
    assert lib.chain_rk4_step(None, 1) == L.CHAIN_EINVAL
    e = ctypes.c_double()
    assert lib.chain_rk4_energy(None, ctypes.byref(e)) == L.CHAIN_EINVAL
    assert lib.chain_rk4_get_plan(None, None) == L.CHAIN_EINVAL
    assert lib.chain_rk4_set_stream(None, None) == L.CHAIN_EINVAL


def test_strerror_covers_all_codes():
    lib = L.lib()
    seen = set()
    for code in (0, -1, -2, -3, -4, -5):
        s = lib.chain_rk4_strerror(code).decode()
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 6
    assert lib.chain_rk4_strerror(12345) == b"unknown status"


def test_oracle_is_not_linked_into_the_product():
    import subprocess
    out = subprocess.run(["nm", "-D", L.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle_" not in out
    src_dir = os.path.join(ROOT, "paper_1412_0544_amd")
    for dirpath, _, files in os.walk(src_dir):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_batch_calls_reject_bad_arguments_without_a_gpu():
    lib = L.lib()
    d = L.BatchDesc(10, 0, 0, 0, 0, 0, 0, 0)
    assert lib.chain_rk4_batch_workspace_bytes(None, 1, ctypes.byref(d)) == 0
    hs = (L.H * 1)(None)
    assert lib.chain_rk4_batch_workspace_bytes(hs, 1, ctypes.byref(d)) == 0
    assert lib.chain_rk4_batch_workspace_bytes(hs, 0, ctypes.byref(d)) == 0
    out = L.VP()
    assert lib.chain_rk4_batch_create(hs, 1, ctypes.byref(d), None, 0, None,
                                      ctypes.byref(out)) == L.CHAIN_EINVAL
    assert lib.chain_rk4_batch_create(hs, 1, None, None, 0, None, ctypes.byref(out)) == L.CHAIN_EINVAL
    assert lib.chain_rk4_batch_step(None, None) == L.CHAIN_EINVAL
    assert lib.chain_rk4_batch_check(None) == L.CHAIN_EINVAL
    assert lib.chain_rk4_batch_destroy(None) == L.CHAIN_OK
    assert lib.chain_rk4_strerror(L.CHAIN_ETIMEOUT) != b"unknown status"


def test_batch_cluster_count_helper():
    from paper_1412_0544_amd.batch import Batch
    lib = L.lib()
    assert lib.chain_rk4_batch_clusters(300, 0, 0) == 1         # a short ring: one cluster

    def wide_only(n, sites, depth):
        keep = 64 * sites * 4 - 4 * depth                          # cluster minus both halos
        return -(-(n // 4) // (keep // 4 - 1))

    for n in (1000, 1025, 5000, 65536, 1 << 24):
        for s, k in ((0, 0), (8, 12), (8, 32)):
            count = lib.chain_rk4_batch_clusters(n, s, k)
            assert count == len(Batch.layout(n, s, k))
            only = Batch.layout(n, s, k, L.CHAIN_BATCH_WIDE_ONLY)
            assert len(only) == wide_only(n, s or 8, k or 32) <= count
    assert lib.chain_rk4_batch_clusters(100, 5, 0) == 0          # invalid shape
    assert lib.chain_rk4_batch_rebind(None, None, 0) == L.CHAIN_EINVAL


def test_roessler_arguments_are_validated_without_a_gpu():
    lib = L.lib()
    f = lambda d: lib.chain_rk4_workspace_bytes(ctypes.byref(d))
    n = 1 << 20
    # fused: three back-buffer arrays; naive: k1..k3 and two stage arguments
    # for each of the three coordinates
    assert f(desc(n=n, model=L.CHAIN_ROESSLER)) >= 3 * 8 * n
    assert f(desc(n=n, model=L.CHAIN_ROESSLER, method=1)) >= 15 * 8 * n
    assert f(desc(n=n, model=L.CHAIN_ROESSLER, prec=1)) == 0       # FP64 only
    h = L.H()
    fake = 1 << 20
    d = desc(model=L.CHAIN_ROESSLER)
    ws = f(d)
    # the two-pointer entry point cannot describe three coordinates
    assert lib.chain_rk4_create(ctypes.byref(d), fake, fake, fake, ws, None,
                                ctypes.byref(h)) == L.CHAIN_EINVAL
    assert b"create3" in lib.chain_rk4_last_error()
    cases = [
        (d, fake, fake, None, ws, L.CHAIN_EINVAL),          # z missing
        (d, fake, fake, fake + 8, ws, L.CHAIN_EINVAL),      # z misaligned
        (d, fake, fake, fake, ws - 1, L.CHAIN_ENOMEM),
        (desc(), fake, fake, fake, f(desc()), L.CHAIN_EINVAL),  # z given to a 2-coordinate model
    ]
    for dd, x, y, z, nb, want in cases:
        assert lib.chain_rk4_create3(ctypes.byref(dd), x, y, z, fake, nb, None,
                                     ctypes.byref(h)) == want


def test_nnn_models_validate_like_the_nn_models():
    lib = L.lib()
    f = lambda d: lib.chain_rk4_workspace_bytes(ctypes.byref(d))
    for m in (L.CHAIN_QUARTIC_NNN, L.CHAIN_HARMONIC_NNN):
        for prec in (0, 1):
            for method in (0, 1):
                assert f(desc(model=m, prec=prec, method=method)) == \
                    f(desc(model=0, prec=prec, method=method))
    assert f(desc(model=3, kdepth=32)) > 0
    h = L.H()
    fake = 1 << 20
    d = desc(model=L.CHAIN_QUARTIC_NNN)
    assert lib.chain_rk4_create(ctypes.byref(d), fake, None, fake, f(d), None,
                                ctypes.byref(h)) == L.CHAIN_EINVAL


def test_tableau_reach_without_a_gpu():
    """The library's reach of one step, for literature tableaus written out
    in the oracle's pin file, equals the reach measured on the oracle there
    (its exact-reach pin) for the NN and NNN chains."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_oracle_tableau import TABLEAUS, step_reach
    from paper_1412_0544_amd.chain import make_tableau
    lib = L.lib()
    for name, ((a, b), _) in TABLEAUS.items():
        t = make_tableau(a.tolist(), b.tolist())
        for model, rng in ((L.CHAIN_QUARTIC, 1), (L.CHAIN_HARMONIC, 1), (L.CHAIN_QUARTIC_NNN, 2)):
            assert lib.chain_rk4_tableau_reach(model, ctypes.byref(t)) == step_reach(a, b, rng), name
    (a, b), _ = TABLEAUS["rk4"]
    t = make_tableau(a.tolist(), b.tolist())
    assert lib.chain_rk4_tableau_reach(L.CHAIN_QUARTIC, ctypes.byref(t)) == 2
    assert lib.chain_rk4_tableau_reach(L.CHAIN_ROESSLER, ctypes.byref(t)) == -1
    t.stages = 9
    assert lib.chain_rk4_tableau_reach(L.CHAIN_QUARTIC, ctypes.byref(t)) == -1
    t.stages = 2
    t.a[1][0] = float("nan")
    assert lib.chain_rk4_tableau_reach(L.CHAIN_QUARTIC, ctypes.byref(t)) == -1
    assert lib.chain_rk4_set_tableau(None, ctypes.byref(t)) == L.CHAIN_EINVAL


def test_preset_tableaus_are_the_literature_values():
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import numpy as np
    from test_oracle_tableau import TABLEAUS
    from paper_1412_0544_amd import tableaus
    assert set(tableaus.ALL) == set(TABLEAUS)
    for name, (a, b) in tableaus.ALL.items():
        (a0, b0), _ = TABLEAUS[name]
        assert np.array_equal(np.array(a), a0) and np.array_equal(np.array(b), b0), name


def test_six_sites_per_lane_only_where_it_is_built():
    """6 sites per lane: the fused classical RK4 of the FP64 quartic and
    harmonic chains and the Roessler chain (fused and exchange form); every
    other descriptor is refused before any HIP call."""
    lib = L.lib()
    ok = [desc(sites_per_lane=6), desc(model=L.CHAIN_HARMONIC, sites_per_lane=6),
          desc(model=L.CHAIN_ROESSLER, sites_per_lane=6),
          desc(n=20000, model=L.CHAIN_ROESSLER, sites_per_lane=6, flags=L.CHAIN_FLAG_EXCHANGE)]
    bad = [desc(prec=L.CHAIN_FP32_KAHAN, sites_per_lane=6),
           desc(prec=L.CHAIN_FP32, sites_per_lane=6),
           desc(model=L.CHAIN_QUARTIC_NNN, sites_per_lane=6),
           desc(sites_per_lane=6, method=L.CHAIN_NAIVE),
           desc(sites_per_lane=6, scheme=L.CHAIN_SCHEME_TABLEAU),
           desc(sites_per_lane=5), desc(sites_per_lane=12)]
    for d in ok:
        assert lib.chain_rk4_workspace_bytes(ctypes.byref(d)) > 0
        P = L.Plan()
        assert lib.chain_rk4_plan_for(ctypes.byref(d), None, ctypes.byref(P)) == L.CHAIN_OK
        assert P.sites_per_lane == 6
    for d in bad:
        assert lib.chain_rk4_workspace_bytes(ctypes.byref(d)) == 0
