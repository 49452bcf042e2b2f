"""The fixed-length line transforms of the momentum-space kernels (radix 2 and 3,
compile-time twiddles), run on the CPU: hipcc builds tests/host/line_fft_check.cpp for
the host, which compares every instantiated length, both signs and both precisions with a
direct DFT in long double (the discrete Fourier transform's definition)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("hipcc not available")


def test_line_fft_matches_direct_dft(tmp_path):
    csrc = os.path.join(ROOT, "paper_1005_3276_amd", "csrc")
    exe = str(tmp_path / "line_fft_check")
    subprocess.run([_hipcc(), "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I", csrc, os.path.join(ROOT, "tests", "host", "line_fft_check.cpp"),
                    "-o", exe], check=True, capture_output=True, text=True, timeout=600)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "line_fft ok" in r.stdout
