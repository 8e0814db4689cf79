"""The C ABI from a plain C program (tests/c_client/client.c, built with gcc
by the build step): no Python and no torch on the device side. Its result
matches the oracle on the same initial state."""
import os
import subprocess

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "chain_client")


def test_c_client_matches_oracle():
    assert os.path.exists(EXE), f"{EXE} is missing: run __graft_entry__.build()"
    n, steps, dt = 5003, 100, 0.01
    out = subprocess.run([EXE, str(n), str(steps), str(dt)], capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    lines = dict((l.split()[0] + (l.split()[1] if l.startswith("site") else ""), l.split())
                 for l in out.stdout.splitlines())
    i = np.arange(n, dtype=np.float64)
    q0 = 0.8 * np.sin(0.37 * i + 0.1)
    p0 = 0.5 * np.cos(0.21 * i)
    qo, po = oracle.rk4(oracle.QUARTIC, q0, p0, dt, steps, threads=8)
    e0 = oracle.energy(oracle.QUARTIC, q0, p0)
    e1 = oracle.energy(oracle.QUARTIC, qo, po)
    assert abs(float(lines["energy0"][1]) - e0) <= 1e-12 * abs(e0)
    assert abs(float(lines["energy"][1]) - e1) <= 1e-12 * abs(e1)
    for s in (0, 1, n // 2, n - 1):
        _, _, q, p = lines[f"site{s}"]
        assert abs(float(q) - qo[s]) <= 1e-10 and abs(float(p) - po[s]) <= 1e-10, s
