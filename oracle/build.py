"""Build the CPU oracle library (test infrastructure only).

Compiles ``rfp_oracle.c`` (real symmetric) and ``zrfp_oracle.c`` (complex
Hermitian) with gcc into ``liboracle_rfp.so`` next to them.
OpenMP only splits independent rows of one column; results do not depend on
the thread count.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "rfp_oracle.c"), os.path.join(HERE, "zrfp_oracle.c")]
LIB = os.path.join(HERE, "liboracle_rfp.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
           "-Wall", "-Wextra", "-Wno-unused-parameter",
           *SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
