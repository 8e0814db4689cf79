"""Explicit Runge-Kutta methods given by their Butcher tableau, on the GPU
against the oracle's general stepper, through the C ABI.

FP64 bar: max-abs state error <= 1e-10 after 100 steps, energy within 1e-12
relative. The tableau kernel gives the same bits at every cluster shape and
depth. The tableaus are the literature values written out in the oracle's
pin file.
"""
import ctypes
import functools
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1412_0544_amd import Chain, ChainError
from paper_1412_0544_amd import _lib as L

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_oracle_tableau import TABLEAUS, step_reach  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-10
OMODEL = {"quartic": oracle.QUARTIC, "harmonic": oracle.HARMONIC,
          "quartic_nnn": oracle.QUARTIC_NNN, "harmonic_nnn": oracle.HARMONIC_NNN}


def tableau(name):
    (a, b), _ = TABLEAUS[name]
    return a.tolist(), b.tolist()


def gpu_run(q0, p0, dt, steps, name, **kw):
    ch = Chain(q0, p0, dt, tableau=tableau(name), **kw)
    ch.step(steps)
    e = ch.energy()
    q, p = (t.cpu().numpy() for t in ch.state())
    plan = ch.plan()
    ch.close()
    return q, p, e, plan


@functools.lru_cache(maxsize=None)
def oracle_run(model, name, n, seed, dt, steps):
    q0, p0 = workloads.chain_ics(n, seed)
    (a, b), _ = TABLEAUS[name]
    return oracle.rk_tableau(OMODEL[model], q0, p0, dt, steps, a, b, threads=8)


def maxerr(a, b):
    return float(np.max(np.abs(a - b))) if a.size else 0.0


def shapes(name):
    s = TABLEAUS[name][0][1].size
    out = [(4, 1), (4, 4)]
    if s <= 4:
        out += [(8, 1), (8, 4)]
    return out


@pytest.mark.parametrize("name", sorted(TABLEAUS))
@pytest.mark.parametrize("model", ["quartic", "quartic_nnn"])
@pytest.mark.parametrize("n", [1, 3, 257, 5003, 20011])
def test_matches_oracle(name, model, n):
    q0, p0 = workloads.chain_ics(n, 1)
    qo, po = oracle_run(model, name, n, 1, 0.01, 100)
    eo = oracle.energy(OMODEL[model], qo, po)
    (a, b), _ = TABLEAUS[name]
    reach = step_reach(a, b, 2 if model.endswith("nnn") else 1)
    for s, w in shapes(name):
        q, p, e, plan = gpu_run(q0, p0, 0.01, 100, name, model=model, sites_per_lane=s,
                                waves_per_cluster=w)
        # the reach of the method, rounded up to a whole 16-byte vector (2 FP64 sites)
        assert plan["halo"] == -(-reach * plan["kdepth"] // 2) * 2
        assert maxerr(q, qo) <= TOL and maxerr(p, po) <= TOL, (s, w)
        assert abs(e - eo) <= 1e-12 * abs(eo)


@pytest.mark.parametrize("name", sorted(TABLEAUS))
def test_shapes_and_depths_identical_bits(name):
    n = 30011
    q0, p0 = workloads.chain_ics(n, 2)
    ref = gpu_run(q0, p0, 0.01, 37, name, sites_per_lane=4, waves_per_cluster=1, kdepth=1)
    for s, w in shapes(name):
        for k in (2, 5, 16, 32):
            got = gpu_run(q0, p0, 0.01, 37, name, sites_per_lane=s, waves_per_cluster=w, kdepth=k)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (s, w, k)
    # the library's plan for chains up to 2^18 sites: one wavefront of 4 per lane
    got = gpu_run(q0, p0, 0.01, 37, name)
    assert (got[3]["sites_per_lane"], got[3]["waves_per_cluster"]) == (4, 1)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("model", ["harmonic", "harmonic_nnn"])
def test_harmonic_models(model):
    n = 4099
    q0, p0 = workloads.chain_ics(n, 3)
    for name in ("kutta3", "dopri5"):
        q, p, e, _ = gpu_run(q0, p0, 0.05, 100, name, model=model)
        qo, po = oracle_run(model, name, n, 3, 0.05, 100)
        assert maxerr(q, qo) <= TOL and maxerr(p, po) <= TOL


def test_fp32_kahan_error_bound():
    n = 20011
    q0, p0 = workloads.chain_ics(n, 4, dtype=np.float32)
    (a, b), _ = TABLEAUS["rk4_38"]
    ch = Chain(q0, p0, 0.01, prec="fp32_kahan", tableau=(a.tolist(), b.tolist()))
    ch.step(100)
    cq, cp = ch.carry_tensors()
    q = (ch.q.double() - cq.double()).cpu().numpy()
    p = (ch.p.double() - cp.double()).cpu().numpy()
    ch.close()
    qo, po = oracle.rk_tableau(oracle.QUARTIC, q0.astype(np.float64), p0.astype(np.float64),
                               0.01, 100, a, b, threads=8)
    err = max(maxerr(q, qo), maxerr(p, po))
    print("tableau fp32_kahan err100", err)
    assert err <= 5e-7


@pytest.mark.parametrize("name", ["rk4", "rk4_38", "kutta3"])
def test_fp32_kahan_drift_tracks_fp64(name):
    """10^4 steps of dt = 0.01 (no FP32 number) from the same FP32-rounded
    state, N = 2^20: the compensated form drifts as FP64 does. Its stage
    arguments take h c_j in two parts, with the increment added to q last;
    with h c_j rounded once every stage argument is offset alike, and the
    energy gains a term of the same sign in every step."""
    n, dt, steps = 1 << 20, 0.01, 10_000
    q, p = workloads.chain_ics_torch(n, 3, "cuda", torch.float32)
    drifts = {}
    for prec, qq, pp in (("fp64", q.double(), p.double()), ("fp32_kahan", q, p)):
        ch = Chain(qq, pp, dt, prec=prec, tableau=tableau(name))
        e0 = ch.energy()
        ch.step(steps)
        drifts[prec] = (ch.energy() - e0) / e0
        ch.close()
    print(name, "drifts", drifts)
    assert drifts["fp64"] < 0, drifts
    assert abs(drifts["fp32_kahan"] / drifts["fp64"] - 1) < 0.03, drifts


def test_tableau_switch_split_calls_and_graphs():
    n = 9000
    q0, p0 = workloads.chain_ics(n, 5)
    (a3, b3), _ = TABLEAUS["kutta3"]
    (a5, b5), _ = TABLEAUS["dopri5"]
    ref = oracle.rk_tableau(oracle.QUARTIC, *oracle.rk_tableau(oracle.QUARTIC, q0, p0, 0.01, 20,
                                                              a3, b3), 0.01, 30, a5, b5)
    for graph in (False, True):
        ch = Chain(q0, p0, 0.01, tableau=(a3.tolist(), b3.tolist()), graph=graph)
        ch.step(7)
        ch.step(13)
        ch.set_tableau(a5.tolist(), b5.tolist())
        ch.step(30)
        torch.cuda.synchronize()
        assert maxerr(ch.q.cpu().numpy(), ref[0]) <= TOL, graph
        assert maxerr(ch.p.cpu().numpy(), ref[1]) <= TOL, graph
        ch.close()


def test_errors():
    q0, p0 = workloads.chain_ics(1000, 6)
    ch = Chain(q0, p0, 0.01)                               # classical scheme
    with pytest.raises(ChainError):
        ch.set_tableau(*tableau("kutta3"))
    ch.close()
    desc = L.Desc(1000, 0, 0, 0.01, 0, 0, 0, 0, 0, L.CHAIN_SCHEME_TABLEAU)
    lib = L.lib()
    ws = lib.chain_rk4_workspace_bytes(ctypes.byref(desc))
    q = torch.from_numpy(q0).cuda()
    p = torch.from_numpy(p0).cuda()
    buf = torch.empty(ws + 256, dtype=torch.uint8, device="cuda")
    ptr = buf.data_ptr() + (-buf.data_ptr()) % 256
    h = L.H()
    assert lib.chain_rk4_create(ctypes.byref(desc), q.data_ptr(), p.data_ptr(), ptr, ws, None,
                                ctypes.byref(h)) == L.CHAIN_OK
    assert lib.chain_rk4_step(h, 1) == L.CHAIN_EINVAL      # no tableau yet
    lib.chain_rk4_destroy(h)
    with pytest.raises(ChainError):                        # 16 sites per lane: not built
        Chain(q0, p0, 0.01, sites_per_lane=16, tableau=tableau("kutta3"))
    with pytest.raises(ChainError):                        # 6 stages need 4 sites per lane
        Chain(q0, p0, 0.01, sites_per_lane=8, tableau=tableau("dopri5"))


def test_large_chain_sampled_sites():
    """N = 2^22, the fifth-order method at the default plan, 100 steps:
    sampled sites against the oracle on windows wider than the light cone."""
    n, steps = 1 << 22, 100
    q0, p0 = workloads.chain_ics(n, 0)
    (a, b), _ = TABLEAUS["dopri5"]
    q, p, _, plan = gpu_run(q0, p0, 0.01, steps, "dopri5")
    r = step_reach(a, b, 1) * steps
    rng = np.random.default_rng(5)
    tile = plan["tile"]
    sites = np.unique(np.concatenate([[0, n - 1, tile - 1, tile], rng.integers(0, n, 12)]))
    for i in sites:
        idx = np.arange(i - r, i + r + 1) % n
        qw, pw = oracle.rk_tableau(oracle.QUARTIC, q0[idx], p0[idx], 0.01, steps, a, b)
        assert abs(q[i] - qw[r]) <= TOL and abs(p[i] - pw[r]) <= TOL, i


@pytest.mark.parametrize("name", sorted(TABLEAUS) + ["euler"])
@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("n", [1, 3, 5003, 300007])
def test_per_stage_path_gives_the_fused_bits(name, prec, n):
    """The one-kernel-per-stage implementation of a tableau method (the
    paper's standard version, Sec. 2.2) and the fused cluster pass give the
    same bits; for FP64 both match the oracle."""
    a, b = ([[0.0]], [1.0]) if name == "euler" else tableau(name)
    dtype = np.float64 if prec == "fp64" else np.float32
    q0, p0 = workloads.chain_ics(n, 7, dtype=dtype)
    outs = []
    for method in ("fused", "naive"):
        ch = Chain(q0, p0, 0.01, prec=prec, method=method, tableau=(a, b))
        ch.step(23)
        cq, cp = ch.carry_tensors()
        outs.append([t.cpu().numpy().copy() for t in
                     (ch.q, ch.p) + ((cq, cp) if cq is not None else ())])
        ch.close()
    for x, y in zip(*outs):
        assert np.array_equal(x, y)
    if prec == "fp64":
        qo, po = oracle.rk_tableau(oracle.QUARTIC, q0, p0, 0.01, 23, np.array(a), np.array(b))
        assert maxerr(outs[0][0], qo) <= TOL and maxerr(outs[0][1], po) <= TOL
