"""Build the FP64 CPU oracle (test infrastructure only).

Compiles ``lgs_oracle.c`` into ``liblgs_oracle.so`` beside it with plain gcc,
no FMA contraction, OpenMP for the per-cell sweep loop.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lgs_oracle.c")
LIB = os.path.join(HERE, "liblgs_oracle.so")


def build(force=True):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
