"""Build step for the oracle's C part (test infrastructure only).

Compiles ``ls_oracle.c`` with gcc into ``liblsoracle.so`` beside it, with
``-ffp-contract=off`` so that every double operation is rounded on its own.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["ls_oracle.c"]
LIB = os.path.join(HERE, "liblsoracle.so")


def compile_library(sources, out, verbose=False):
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", out + ".tmp"]
    cmd += list(sources) + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    return compile_library([os.path.join(HERE, s) for s in SOURCES], LIB, verbose)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
