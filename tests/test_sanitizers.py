"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code, on
the CPU: the oracle (every entry point on small rings) and the library's
host translation units (planning, workspace layout, argument validation and
the batch bookkeeping) with the kernel launchers stubbed out. Any finding
aborts the driver, which fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1412_0544_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="abort_on_error=1:detect_leaks=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    run(["gcc", "-std=c99", *SAN, "-fopenmp", "-ffp-contract=off",
         os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "chain_oracle.c"),
         "-o", exe, "-lm"])
    r = run([exe], env=dict(ENV, OMP_NUM_THREADS="3"), timeout=300)
    assert "all calls clean" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or
                    not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")),
                    reason="needs g++ and the HIP headers")
def test_host_library_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    inc = ["-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", f"-I{ROOT}/include", f"-I{CSRC}"]
    objs = []
    for src in (os.path.join(CSRC, "chain_rk4.cpp"), os.path.join(CSRC, "batch.cpp"),
                os.path.join(HERE, "launch_stubs.cpp"), os.path.join(HERE, "host_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        run(["g++", "-std=c++17", *SAN, *inc, "-c", src, "-o", obj])
        objs.append(obj)
    run(["g++", *SAN, *objs, "-o", exe, f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"])
    # the HIP runtime's own start-up allocations are not this code's
    r = run([exe], env=dict(ENV, ASAN_OPTIONS="abort_on_error=1:detect_leaks=0",
                            HIP_VISIBLE_DEVICES=""), timeout=600)
    assert "all invariants hold" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or
                    not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")),
                    reason="needs g++ and the HIP headers")
def test_exchange_bookkeeping_under_sanitizers(tmp_path):
    """The exchange form's pass counters over successive calls (the base each
    launch starts from), with recording launchers in place of the kernels."""
    exe = str(tmp_path / "exchange_driver")
    inc = ["-D__HIP_PLATFORM_AMD__", "-DRECORD_EXCHANGE", f"-I{ROCM}/include",
           f"-I{ROOT}/include", f"-I{CSRC}"]
    objs = []
    for src in (os.path.join(CSRC, "chain_rk4.cpp"), os.path.join(CSRC, "batch.cpp"),
                os.path.join(HERE, "launch_stubs.cpp"), os.path.join(HERE, "exchange_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        run(["g++", "-std=c++17", *SAN, *inc, "-c", src, "-o", obj])
        objs.append(obj)
    run(["g++", *SAN, *objs, "-o", exe, f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"])
    r = run([exe], env=dict(ENV, ASAN_OPTIONS="abort_on_error=1:detect_leaks=0",
                            HIP_VISIBLE_DEVICES=""), timeout=300)
    assert "exchange bookkeeping holds" in r.stdout
