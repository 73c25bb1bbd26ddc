"""Build the CPU oracle's shared library (``liboracle_gf2.so``) with gcc.

Test infrastructure: the product never loads this library.

Two builds of the same source:

* the in-tree library used by the tests, ``-O3`` for the generic x86-64 target, so it runs
  on any host the repository is copied to;
* ``build(native=True, out_dir=...)``, ``-O3 -march=native``, compiled on the host that runs
  it (the benchmark's CPU-baseline leg), into a directory of the caller's choosing.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle_gf2.so")
FLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp"]


def build(verbose: bool = False, native: bool = False, out_dir: str | None = None) -> str:
    src = os.path.join(HERE, "gf2ref.c")
    lib = LIB if out_dir is None else os.path.join(out_dir, "liboracle_gf2.so")
    flags = FLAGS + (["-march=native"] if native else [])
    cmd = ["gcc", *flags, src, "-o", lib + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


def command(native: bool = False) -> str:
    """The gcc command line of a build (for reports)."""
    return " ".join(["gcc", *FLAGS, *(["-march=native"] if native else []), "gf2ref.c"])


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
