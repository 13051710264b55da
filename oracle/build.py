"""Build the CPU oracle library (test infrastructure).

gcc, -O2, no fast-math and no floating-point contraction: every multiply-add
the oracle wants fused is written as fma() in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "mcubes_oracle.c"), os.path.join(HERE, "mcubes_oracle_abi.c"),
        os.path.join(HERE, "flow_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-shared", "-fPIC", "-o", LIB, *SRCS, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
