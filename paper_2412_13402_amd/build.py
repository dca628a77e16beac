"""Build librtbte.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "librtbte.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "diagnostics.hip", "api.hip")]


def hipcc_command(out=LIB, arch="gfx950"):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return [hipcc, "-O3", "-std=c++17", f"--offload-arch={arch}", "-fPIC", "-shared", "-fopenmp",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
            "-o", out] + SOURCES


def build(verbose=False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
