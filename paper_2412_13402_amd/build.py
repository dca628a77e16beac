"""Build librtbte.so (HIP, gfx950) in-tree with hipcc, and the plain-C example
program that uses it (build/example_rhs)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "librtbte.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "diagnostics.hip", "api.hip")]
EXAMPLE = os.path.join(HERE, "build", "example_rhs")


def hipcc_command(out=LIB, arch="gfx950"):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return [hipcc, "-O3", "-std=c++17", f"--offload-arch={arch}", "-fPIC", "-shared", "-fopenmp",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
            "-o", out] + SOURCES + ["-L", os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib"),
                                    "-lrocprofiler-sdk-roctx"]


def example_command(out=EXAMPLE):
    """The C example: a C99 program against include/rtbte.h and the HIP
    runtime's C API, linked to librtbte.so (found next to it at run time)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(rocm, "include"),
            os.path.join(HERE, "csrc", "example_rhs.c"), "-o", out,
            "-L", HERE, "-lrtbte", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
            "-Wl,-rpath,$ORIGIN/..", "-Wl,-rpath," + os.path.join(rocm, "lib")]


def build(verbose=False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    os.makedirs(os.path.dirname(EXAMPLE), exist_ok=True)
    cmd = example_command()
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
