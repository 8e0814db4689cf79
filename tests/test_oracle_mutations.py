"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU),
builds it, and runs the pin suite against that build; at least one pin has to
fail. The unmodified source must pass the same suite.
"""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

MUTANTS = {
    "drop_onsite_cubic": ("return -(q + q * q * q) + dr * dr * dr - dl * dl * dl;",
                          "return -(q) + dr * dr * dr - dl * dl * dl;"),
    "coupling_sign": ("+ dr * dr * dr - dl * dl * dl;", "- dr * dr * dr + dl * dl * dl;"),
    "wrong_neighbour": ("double dl = q - qm;", "double dl = q - qp;"),
    "boundary_wrap": ("return i == 0 ? n - 1 : i - 1;", "return i == 0 ? 0 : i - 1;"),
    "harmonic_laplacian": ("return -q + (qp - 2.0 * q + qm);", "return -q + (qp - q + qm);"),
    "stage2_step": ("intermediate(n, q, p, dt / 2.0, k2q, k2p", "intermediate(n, q, p, dt, k2q, k2p"),
    "stage4_uses_k2": ("intermediate(n, q, p, dt, k3q, k3p", "intermediate(n, q, p, dt, k2q, k2p"),
    "momentum_stage_operand": ("P[i] = p[i] + a_dt * kp[i];", "P[i] = p[i] + a_dt * kq[i];"),
    "weight_k2": ("(k1q[i] + 2.0 * k2q[i]", "(k1q[i] + k2q[i]"),
    "weight_k4_p": ("2.0 * k3p[i] + k4p[i])", "2.0 * k3p[i] + 2.0 * k4p[i])"),
    "final_dt": ("q[i] = q[i] + (dt / 6.0)", "q[i] = q[i] + (dt / 3.0)"),
    "energy_bond": ("+ d * d * d * d / 4.0;", "+ d * d * d * d / 2.0;"),
    "energy_kinetic": ("return p * p / 2.0 + q * q / 2.0 + d * d / 2.0;",
                       "return p * p + q * q / 2.0 + d * d / 2.0;"),
    "roessler_coupling_sign": ("kx[i] = -y[i] - z[i] + (xm - 2.0 * x[i] + xp);",
                               "kx[i] = -y[i] - z[i] - (xm - 2.0 * x[i] + xp);"),
    "roessler_coupling_weight": ("(xm - 2.0 * x[i] + xp)", "(xm - x[i] + xp)"),
    "roessler_y_term": ("ky[i] = x[i] + a * y[i];", "ky[i] = x[i] + a * x[i];"),
    "roessler_z_term": ("kz[i] = b + z[i] * (x[i] - c);", "kz[i] = b + z[i] * (x[i] + c);"),
    "roessler_stage3": ("intermediate3(n, x, y, z, dt, k[2][0]", "intermediate3(n, x, y, z, dt / 2.0, k[2][0]"),
    "roessler_final_z": ("2.0 * k[2][2][i] + k[3][2][i])", "k[2][2][i] + k[3][2][i])"),
    "nnn_drop_second_bonds": (" + dr2 * dr2 * dr2 - dl2 * dl2 * dl2;", ";"),
    "nnn_second_sign": ("+ dr2 * dr2 * dr2 - dl2 * dl2 * dl2", "+ dr2 * dr2 * dr2 + dl2 * dl2 * dl2"),
    "nnn_second_index": ("q[wrap(i, -2, n)], q[left_of(i, n)]", "q[wrap(i, -1, n)], q[left_of(i, n)]"),
    "nnn_harmonic_second": ("(qpp - 2.0 * q + qmm)", "(qpp - q + qmm)"),
    "nnn_wrap": ("return j < 0 ? j + n : j;", "return j < 0 ? 0 : j;"),
    "nnn_energy_second": ("d2 * d2 * d2 * d2 / 4.0", "d2 * d2 * d2 * d2 / 2.0"),
    "nnn_energy_harmonic": ("+ d2 * d2 / 2.0;", "+ d2 * d2;"),
    "tableau_stage_dt": ("Q[i] = q[i] + dt * sq;", "Q[i] = q[i] + sq;"),
    "tableau_transposed": ("sq += a[j * s + m] * kq", "sq += a[m * s + j] * kq"),
    "tableau_momentum_slope": ("sp += a[j * s + m] * kp", "sp += a[j * s + m] * kq"),
    "tableau_stage_count": ("for (m = 0; m < j; ++m) {", "for (m = 0; m + 1 < j; ++m) {"),
    "tableau_weights": ("sq += b[m] * kq[(size_t)m * n + i];", "sq += b[0] * kq[(size_t)m * n + i];"),
    "tableau_final_dt": ("p[i] = p[i] + dt * sp;", "p[i] = p[i] + 0.5 * dt * sp;"),
}


def _run_pins(lib):
    env = dict(os.environ, CHAIN_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_pins.py"),
                        os.path.join(HERE, "test_oracle_roessler.py"),
                        os.path.join(HERE, "test_oracle_nnn.py"),
                        os.path.join(HERE, "test_oracle_tableau.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    return r.returncode


def test_unmodified_oracle_passes_pins(tmp_path):
    lib = oracle.build(force=True, src=oracle.SRC, out=str(tmp_path / "lib_ok.so"))
    assert _run_pins(lib) == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {old!r}"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = oracle.build(force=True, src=str(path), out=str(tmp_path / "mutant.so"))
    assert _run_pins(lib) != 0, f"no pin caught mutant {name}"
