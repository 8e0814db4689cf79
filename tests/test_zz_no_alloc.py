"""The entry point that allocates nothing: chain_rk4_energy_noalloc, called
through the C ABI, gives the same bits as chain_rk4_energy of a handle over
the same state, on two calls in a row (the second with a smaller input, so
stale partial sums of the first would show), and rejects sizes beyond its
limit."""
import ctypes

import numpy as np
import pytest
import torch

import workloads
from paper_1412_0544_amd import Chain
from paper_1412_0544_amd import _lib as L
from paper_1412_0544_amd.chain import MODELS, PRECS

pytestmark = pytest.mark.gpu


def noalloc(model, prec, q, p, cq=None, cp=None, n=None):
    ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
    e = ctypes.c_double(0.0)
    stream = torch.cuda.current_stream().cuda_stream
    rc = L.lib().chain_rk4_energy_noalloc(MODELS[model], PRECS[prec],
                                          q.numel() if n is None else n, ptr(q), ptr(p), ptr(cq),
                                          ptr(cp), stream, ctypes.byref(e))
    return rc, e.value


def stepped_chain(n, seed, model, prec, steps=60):
    dtype = np.float64 if prec == "fp64" else np.float32
    q0, p0 = workloads.chain_ics(n, seed, dtype=dtype)
    ch = Chain(q0, p0, 0.01, model=model, prec=prec)
    ch.step(steps)
    return ch


@pytest.mark.parametrize("model", ["quartic", "harmonic_nnn"])
@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan", "fp32_kahan64", "fp32"])
def test_noalloc_energy_equals_the_handle_energy_twice(model, prec):
    for n in (1_000_003, 4097):            # the second call is smaller
        ch = stepped_chain(n, 3, model, prec)
        want = ch.energy()
        cq, cp = ch.carry_tensors()
        rc, got = noalloc(model, prec, ch.q, ch.p, cq, cp)
        assert rc == L.CHAIN_OK
        assert got == want, (n, got, want)                # same kernels, same bits
        ch.close()


def test_noalloc_limits_and_arguments():
    ch = stepped_chain(1000, 1, "quartic", "fp64")
    q, p = ch.q, ch.p
    for n in (0, -5, (1 << 40) + 1):
        assert noalloc("quartic", "fp64", q, p, n=n)[0] == L.CHAIN_EINVAL
    assert b"2^40" in L.lib().chain_rk4_last_error()
    assert noalloc("quartic", "fp64", q, p, q, p)[0] == L.CHAIN_EINVAL    # carries with FP64
    k = stepped_chain(1000, 1, "quartic", "fp32_kahan")
    assert noalloc("quartic", "fp32_kahan", k.q, k.p)[0] == L.CHAIN_EINVAL  # carries missing
    rc = L.lib().chain_rk4_energy_noalloc(L.CHAIN_ROESSLER, 0, 1000, q.data_ptr(), p.data_ptr(),
                                          None, None, None, ctypes.byref(ctypes.c_double()))
    assert rc == L.CHAIN_EINVAL
    # a state that is not finite: CHAIN_ENONFINITE with the value written
    q[10] = float("nan")
    rc, e = noalloc("quartic", "fp64", q, p)
    assert rc == L.CHAIN_ENONFINITE and np.isnan(e)
    ch.close()
    k.close()
