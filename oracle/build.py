"""Build the CPU oracle shared library (test infrastructure).

Compiles ``bgk_oracle.c`` with gcc into ``liboracle.so`` next to this file.
Portable flags only (no -march=native, no -ffast-math): the library built here
must also run on other x86-64 hosts and keep IEEE semantics.  ``build_native``
compiles the same source with -O3 -march=native (still no -ffast-math) for the
host it runs on; the benchmark's CPU-baseline leg times that build.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bgk_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, out: str = LIB, opt=("-O2",)) -> str:
    tmp = out + ".tmp"
    cmd = ["gcc", *opt, "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
           "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_native(out: str, verbose: bool = False) -> str:
    """The oracle tuned for this host's CPU (-O3 -march=native); built where
    it runs, never shipped."""
    return build(verbose, out=out, opt=("-O3", "-march=native"))


if __name__ == "__main__":
    print(build(verbose=True))
