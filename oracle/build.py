"""Build the plain C oracle (liboracle.so) beside this file.

Portable flags only (-O2 -mpopcnt, no -march=native): the library is built in
one place and may run on another host CPU.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chm_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-mpopcnt", "-fopenmp", "-std=c11", "-Wall", "-Wextra",
           "-shared", "-fPIC", SRC, "-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
