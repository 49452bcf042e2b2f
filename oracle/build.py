"""Build step for the CPU oracle (test infrastructure).

Compiles ``ov_oracle.c`` with gcc (-O2, AVX2/FMA, OpenMP over site loops) into
``libovoracle.so`` beside this file.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libovoracle.so")


def build(verbose: bool = False) -> str:
    # -march=x86-64-v3 (AVX2 + FMA) rather than -march=native: the library built here is
    # also loaded on other hosts, whose CPUs may lack this one's newer extensions.  -O2, not
    # -O3: -O3's loop vectoriser makes the complex site loops slower (MdagM at 16^4 on 8
    # threads: -O2 2.2 s, -O3 4.3 s, -O2 -march=x86-64-v3 2.0 s)
    cmd = ["gcc", "-O2", "-march=x86-64-v3", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wno-unused-variable",
           os.path.join(HERE, "ov_oracle.c"), "-o", SO + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(SO + ".tmp", SO)
    return SO


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
