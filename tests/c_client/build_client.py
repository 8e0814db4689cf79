"""Compile the plain C client of the library (gcc, HIP runtime C API)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
EXE = os.path.join(HERE, "chain_client")


def build() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    lib_dir = os.path.join(ROOT, "paper_1412_0544_amd")
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROOT}/include", f"-I{rocm}/include", os.path.join(HERE, "client.c"),
           "-o", EXE, f"-L{lib_dir}", "-lchainrk4", "-Wl,-rpath,$ORIGIN/../../paper_1412_0544_amd",
           f"-L{rocm}/lib", "-lamdhip64", f"-Wl,-rpath,{rocm}/lib", "-lm"]
    subprocess.run(cmd, check=True)
    return EXE


if __name__ == "__main__":
    print(build())
