"""Compile the C part of the oracle (test infrastructure only).

``python -m oracle.build`` or ``oracle.build.build()`` produces
``oracle/libmd_oracle.so`` with gcc, FP64, no FMA contraction, no fast-math,
OpenMP over atoms in the force loop.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "md_oracle.c")
LIB = os.path.join(HERE, "libmd_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
