"""Build the CPU oracle's shared library (plain C, gcc).

The oracle is test infrastructure: only the tests, the smoke check and the
benchmark's CPU-baseline leg load it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["oracle.c", "snn.c", "proj.c"]
LIB = os.path.join(HERE, "liboracle.so")
# the same sources with their OpenMP pragmas honoured: the network loops
# spread over the host cores (the CPU baseline); results are identical
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def _gcc(out, extra, verbose):
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    # -ffp-contract=off: every FP32 operation of the network recursion is
    # rounded on its own, in program order (no fused multiply-add).
    cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", *extra,
           "-o", out + ".tmp", *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False) -> str:
    _gcc(LIB, [], verbose)
    _gcc(LIB_OMP, ["-fopenmp"], verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
