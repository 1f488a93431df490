"""Build the CPU oracle shared library (test infrastructure).

Compiles ``bgk_oracle.c`` with gcc into ``liboracle.so`` next to this file.
Portable flags only (no -march=native, no -ffast-math): the library built here
must also run on other x86-64 hosts and keep IEEE semantics.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bgk_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
           "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
