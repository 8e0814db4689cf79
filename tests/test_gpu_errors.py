"""Error paths on the GPU, through the C ABI: a state that is not finite makes
the energy calls return CHAIN_ENONFINITE (with the value written), for single
chains and for every chain of a batch, without disturbing the other chains."""
import ctypes
import math

import numpy as np
import pytest
import torch

import workloads
from paper_1412_0544_amd import Batch, Chain, ChainError
from paper_1412_0544_amd import _lib as L

pytestmark = pytest.mark.gpu


def raw_energy(ch):
    e = ctypes.c_double(0.0)
    rc = L.lib().chain_rk4_energy(ch.handle, ctypes.byref(e))
    return rc, e.value


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan", "fp32_kahan64", "fp32"])
@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_energy_of_a_nonfinite_state(prec, bad):
    n = 3001
    dtype = np.float64 if prec == "fp64" else np.float32
    q0, p0 = workloads.chain_ics(n, 5, dtype=dtype)
    good = Chain(q0, p0, 0.01, prec=prec)
    rc, e = raw_energy(good)
    assert rc == L.CHAIN_OK and math.isfinite(e)
    for arr in ("q", "p"):
        ch = Chain(q0, p0, 0.01, prec=prec)
        getattr(ch, arr)[1234] = bad
        rc, e = raw_energy(ch)
        assert rc == L.CHAIN_ENONFINITE and not math.isfinite(e), (arr, rc, e)
        assert b"not finite" in L.lib().chain_rk4_last_error()
        with pytest.raises(ChainError) as ex:
            ch.energy()
        assert ex.value.status == L.CHAIN_ENONFINITE
        # the value spreads through the ring as the chain is stepped; the
        # energy call keeps reporting it
        ch.step(40)
        rc, e = raw_energy(ch)
        assert rc == L.CHAIN_ENONFINITE
        ch.close()
    good.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_batch_energy_reports_the_nonfinite_chain_and_fills_the_rest(prec):
    dtype = np.float64 if prec == "fp64" else np.float32
    lengths = [500, 20011, 3000]
    chains = [Chain(*workloads.chain_ics(n, 40 + i, dtype=dtype), 0.01, prec=prec)
              for i, n in enumerate(lengths)]
    b = Batch(chains, max_steps=64)
    b.step([64, 64, 64])
    b.check()
    want = [c.energy() for c in chains]
    chains[1].q[777] = float("nan")
    torch.cuda.synchronize()
    out = (ctypes.c_double * 3)()
    rc = L.lib().chain_rk4_batch_energy(b._b, out)
    assert rc == L.CHAIN_ENONFINITE
    assert out[0] == want[0] and out[2] == want[2]
    assert math.isnan(out[1])
    with pytest.raises(ChainError) as ex:
        b.energies()
    assert ex.value.status == L.CHAIN_ENONFINITE
    b.close()
    for c in chains:
        c.close()
