"""Builds the C oracle into ``oracle/libttxref.so`` with gcc.

Test infrastructure: the oracle is compiled so that the tests, the smoke
check and the benchmark's CPU-baseline leg can load it; the library under
test never does.  Floating-point contraction is switched off and no
fast-math flag is given, so every product and sum is rounded on its own in
the element type (IEEE round-to-nearest, subnormals kept).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ttx_ref.c")
LIB = os.path.join(HERE, "libttxref.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(out=LIB, src=SRC, extra=()):
    """Compiles ``src`` to the shared library ``out``; returns ``out``."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", *CFLAGS, *extra, "-o", tmp, src], check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
