"""Build step for the oracle's C part (test infrastructure only).

Compiles ``oracle/c/oracle_fft.c`` with plain gcc into ``oracle/c/liboracle.so``.
IEEE semantics are kept (no -ffast-math) so that results do not depend on
reassociation.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "oracle_fft.c")
LIB = os.path.join(HERE, "c", "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
