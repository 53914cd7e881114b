"""Build the oracle's shared object with gcc (test infrastructure only).

The flags keep binary64 arithmetic exactly as written: no fast-math, no FMA
contraction, so the reference is reproducible across hosts.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "fip_oracle.c"), os.path.join(HERE, "fip_oracle_mx.c"),
        os.path.join(HERE, "fip_oracle_l3.c"), os.path.join(HERE, "fip_oracle_cx.c")]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", *SRCS, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
