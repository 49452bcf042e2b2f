"""Build step for the CPU oracle (test infrastructure).

Compiles ``ov_oracle.c`` with gcc into ``libovoracle.so`` beside this file.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libovoracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wno-unused-variable",
           os.path.join(HERE, "ov_oracle.c"), "-o", SO + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(SO + ".tmp", SO)
    return SO


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
