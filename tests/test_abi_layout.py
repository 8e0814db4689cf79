"""The ctypes mirrors of the C structs have the C layout (checked by compiling
the header with the host C compiler)."""
import ctypes
import os
import subprocess

from paper_1412_0544_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include <stddef.h>
#include <stdio.h>
#include "chain_rk4.h"
#define F(T, m) printf("%s.%s %zu\n", #T, #m, offsetof(T, m));
int main(void) {
  %FIELDS%
  return 0;
}
"""


STRUCTS = (("chain_rk4_desc", L.Desc), ("chain_rk4_plan", L.Plan),
           ("chain_rk4_batch_desc", L.BatchDesc), ("chain_rk4_batch_plan", L.BatchPlan),
           ("chain_rk4_tableau", L.Tableau))


def test_struct_layouts_match(tmp_path):
    fields = []
    for cname, cls in STRUCTS:
        fields.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for name, _ in cls._fields_:
            fields.append(f"F({cname}, {name})")
    src = tmp_path / "layout.c"
    src.write_text(PROGRAM.replace("%FIELDS%", "\n  ".join(fields)))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", f"-I{ROOT}/include", str(src), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run(
        [str(exe)], capture_output=True, text=True, check=True).stdout.split("\n") if line)
    for cname, cls in STRUCTS:
        assert int(out[cname]) == ctypes.sizeof(cls), cname
    for cname, cls in STRUCTS:
        for name, _ in cls._fields_:
            assert int(out[f"{cname}.{name}"]) == getattr(cls, name).offset, (cname, name)
