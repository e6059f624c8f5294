"""Build the oracle's shared library with gcc (plain C, FP64, no contraction).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "adr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
         "-shared", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    """Compile ``adr_oracle.c`` into ``liboracle.so`` next to it; return its path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + FLAGS + ["-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
