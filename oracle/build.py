"""Compiles the C oracle into oracle/liboracle.so (test infrastructure).

Plain gcc, -O2, no fast-math and no FMA contraction, so the oracle's
arithmetic is the straightforward IEEE FP64 evaluation of its source.
"""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build():
    src = os.path.join(_HERE, "oracle.c")
    out = os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-Wno-unused-parameter", src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
