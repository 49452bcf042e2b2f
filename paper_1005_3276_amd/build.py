"""Build libov.so (HIP, gfx950) in-tree with hipcc.

Every HIP translation unit is compiled with packed FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libov.so")
ARCH = os.environ.get("OV_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    cc = hipcc()
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
              "-I", os.path.join(HERE, "..", "include")]
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    srcs = [("ov_lib.hip", True), ("ov_zolotarev.cpp", False), ("ov_host.cpp", False)]
    for name, device in srcs:
        src = os.path.join(CSRC, name)
        obj = os.path.join(build_dir, name + ".o")
        cmd = [cc] + common + ["-c", src, "-o", obj]
        if device:
            cmd[1:1] = ["-x", "hip", f"--offload-arch={ARCH}",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    link = ([cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", SO + ".tmp"] + objs +
            ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"])
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(SO + ".tmp", SO)
    return SO


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
