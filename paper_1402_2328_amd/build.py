"""Build librewl.so (HIP, gfx950) in-tree.

Flags that matter for results:
  -ffp-contract=off      no implicit multiply-add fusion: every FMA in the
                         kernels is written explicitly, so floating-point
                         results are defined by the source;
  -fhip-fp32-correctly-rounded-divide-sqrt
                         IEEE single-precision division (two-float merge);
  -Xclang -target-feature -Xclang -packed-fp32-ops
                         keeps the compiler from forming packed FP32 ops.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librewl.so")
ALU_LIB = os.path.join(HERE, "libalurate.so")
SOURCES = ["rewl_sweep.hip", "rewl_kernels.hip", "rewl_api.cpp", "rewl_plan.cpp"]
ARCH = os.environ.get("REWL_OFFLOAD_ARCH", "gfx950")


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
            "-fhip-fp32-correctly-rounded-divide-sqrt",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I", os.path.join(os.path.dirname(HERE), "include")]


def build(verbose=False):
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(bdir, src.rsplit(".", 1)[0] + ".o")
        cmd = [hipcc(), *flags(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc(), "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    build_alu_rate(verbose)
    return LIB


def build_alu_rate(verbose=False):
    """libalurate.so: the instruction issue-cost probe behind the sweep's roofline."""
    tmp = ALU_LIB + ".tmp"
    cmd = [hipcc(), *flags(), "-shared", "-x", "hip", os.path.join(CSRC, "alu_rate.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, ALU_LIB)
    return ALU_LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
