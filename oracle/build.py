"""Build the oracle shared libraries (test infrastructure only).

Two builds of the one source file ``pw_oracle.c``:
  * ``libpworacle.so``      single-threaded, the reference for parity tests;
  * ``libpworacle_omp.so``  the same source with ``-fopenmp`` (only the forward
    loop is threaded), used for the multithreaded host baseline.

Both are built with ``-O2 -ffp-contract=off -fno-fast-math`` so that every
operation is rounded exactly once in the order the source states.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pw_oracle.c")
FLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC"]


def build_oracle(verbose=False):
    outs = []
    for name, extra in (("libpworacle.so", []), ("libpworacle_omp.so", ["-fopenmp"])):
        out = os.path.join(HERE, name)
        cmd = ["gcc"] + FLAGS + extra + [SRC, "-o", out + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
        outs.append(out)
    return outs


if __name__ == "__main__":
    for p in build_oracle(verbose=True):
        print(p)
