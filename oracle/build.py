"""Compiles the C oracle (test infrastructure).

liboracle.so, the build the tests load: plain gcc -O2, no fast-math and no
FMA contraction, no OpenMP, so the oracle's arithmetic is the straightforward
IEEE FP64 evaluation of its source in the order written.

liboracle_omp.so, the host-timing build of the same source for the
benchmark's CPU baseline: -O3 for x86-64-v3 (AVX2; any recent x86 host) with OpenMP over the solve's
cell loops (its reductions may sum in another order); still no fast-math
and no contraction.
"""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_COMMON = ["-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-Wno-unused-parameter"]


def _gcc(flags, out):
    src = os.path.join(_HERE, "oracle.c")
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.run(["gcc"] + flags + _COMMON + [src, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, out)
    return out


def build():
    out = _gcc(["-O2", "-Wno-unknown-pragmas"], os.path.join(_HERE, "liboracle.so"))
    _gcc(["-O3", "-march=x86-64-v3", "-fopenmp"], os.path.join(_HERE, "liboracle_omp.so"))
    return out


if __name__ == "__main__":
    print(build())
