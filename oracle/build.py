"""Build the oracle's shared library (plain C, gcc, FP64, no fast-math).

Test infrastructure: the library this builds is loaded only by the test-suite,
the smoke check and the benchmark's CPU-baseline leg.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vsh_oracle.c")
LIB = os.path.join(HERE, "libvsh_oracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]


def build(march_native: bool = False, out: str = LIB) -> str:
    flags = list(CFLAGS)
    if march_native:
        flags[0] = "-O3"
        flags.append("-march=native")
    cmd = ["gcc", *flags, "-o", out + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(march_native="--native" in sys.argv))
