"""Build step for the CPU oracle (test infrastructure): gcc -> oracle/liborc.so.

Strict IEEE evaluation: no FMA contraction, no fast-math.  OpenMP splits
independent items across host threads; libquadmath supplies binary128.
"""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "glv_oracle.c")


def library_path() -> str:
    return os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    out = library_path()
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-Wall", "-Wextra", "-Werror", "-o", tmp, SOURCE, "-lquadmath", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
