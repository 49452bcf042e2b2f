"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code (CPU only):

* the C oracle, every entry point on 2^4 .. 4^4 lattices and every Dirac form
  (tests/sanitize/oracle_check.c);
* libov.so's host-only functions: parameter validation, the free |H_W| spectrum, the CG
  bound and the Zolotarev generator (tests/sanitize/host_check.cpp against
  csrc/ov_host.cpp and csrc/ov_zolotarev.cpp).

Each is built with gcc / g++ -fsanitize=address,undefined and -fno-sanitize-recover, so
any report ends the program with a non-zero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _build_run(cmd, exe, tmp_path, expect):
    if not shutil.which(cmd[0]):
        pytest.skip(f"{cmd[0]} not available")
    out = str(tmp_path / exe)
    subprocess.run(cmd + ["-o", out], check=True, capture_output=True, text=True)
    r = subprocess.run([out], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert expect in r.stdout


def test_oracle_under_sanitizers(tmp_path):
    _build_run(["gcc", "-std=gnu11"] + SAN +
               ["-I", os.path.join(ROOT, "oracle"),
                os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"),
                os.path.join(ROOT, "oracle", "ov_oracle.c"), "-lm"],
               "oracle_check", tmp_path, "oracle_check ok")


def test_library_host_code_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1005_3276_amd", "csrc")
    _build_run(["g++", "-std=c++17"] + SAN +
               ["-I", csrc, os.path.join(ROOT, "tests", "sanitize", "host_check.cpp"),
                os.path.join(csrc, "ov_host.cpp"), os.path.join(csrc, "ov_zolotarev.cpp")],
               "host_check", tmp_path, "host_check ok")
