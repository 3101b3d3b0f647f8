"""Compile the CPU oracle (test infrastructure only).

Two shared libraries are built from the same C sources with gcc:
  liboracle.so     double precision (matrix elements, Philox, RAMBO);
  liboracle_ld.so  long double (x87 80-bit) matrix elements, the referee for events whose
                   double-precision value is ill-conditioned.
No HIP code, header or generated table is involved.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CFLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
          "-Wall", "-Wno-unused-function"]


def build(verbose=False):
    jobs = [
        ("liboracle.so", ["me.c", "rambo.c"], ["-DOR_REAL=double"]),
        ("liboracle_ld.so", ["me.c"], ["-DOR_REAL=long double"]),
    ]
    for out, srcs, defs in jobs:
        cmd = ["gcc"] + CFLAGS + defs + [os.path.join(HERE, s) for s in srcs] + \
              ["-o", os.path.join(HERE, out), "-lm", "-lpthread"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)


if __name__ == "__main__":
    build(verbose=True)
