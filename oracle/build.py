"""Build the reference oracle (test infrastructure only).

Compiles ``rewl_oracle.c`` into ``liboracle.so`` next to this file with gcc,
-O2, no fast-math and no floating-point contraction, so that every
floating-point operation in the oracle is exactly the one written in the C
source.  Only the test-suite, the smoke check and the benchmark's CPU-baseline
leg use the result.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "rewl_oracle.c")

CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
          "-fno-fast-math", "-fPIC", "-shared"]


def build(force=True):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
