"""Host-side checks of libov.so that need no GPU: it loads, exports every
symbol include/ov.h declares, and its host logic (parameter validation, the
spectrum check, the Zolotarev generator) agrees with the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1005_3276_amd import _lib as L
    if not os.path.exists(L.SO):
        pytest.skip("libov.so not built")
    return L


def test_exports_every_declared_symbol():
    L = _lib()
    hdr = open(os.path.join(ROOT, "include", "ov.h")).read()
    declared = set(re.findall(r"\b(ov_[a-z_]+)\s*\(", hdr))
    assert declared, "no declarations parsed"
    lib = L.lib()
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(L.SYMBOLS)


@pytest.mark.parametrize("n,lmin,lmax", [(16, 0.01, 8.0), (20, 1e-3, 8.0), (24, 1e-4, 8.0),
                                         (8, 1.0, 7.0), (1, 0.5, 2.0)])
def test_library_zolotarev_matches_oracle(orc, n, lmin, lmax):
    L = _lib()
    a, b, d = L.zolotarev(n, lmin, lmax)
    a2, b2, d2, _ = orc.zolotarev(n, lmin, lmax)
    assert np.max(np.abs(a / a2 - 1)) < 1e-12
    assert np.max(np.abs(b / b2 - 1)) < 1e-12
    assert abs(d - d2) < 1e-14 + 1e-6 * d2


def _create(**kw):
    L = _lib()
    p = L.default_params(**kw)
    h = C.c_void_p()
    st = L.lib().ov_ctx_create(C.byref(p), None, C.byref(h))
    if st == L.OV_OK:
        L.lib().ov_ctx_destroy(h)
    return st


def test_ctx_create_rejects_bad_params():
    L = _lib()
    assert _create(dims=(3, 4, 4, 4)) == L.OV_ERR_INVALID_ARG      # odd extent
    assert _create(dims=(4, 4, 4, 0)) == L.OV_ERR_INVALID_ARG      # empty lattice
    assert _create(n_poles=0) == L.OV_ERR_INVALID_ARG
    assert _create(n_poles=33) == L.OV_ERR_INVALID_ARG
    assert _create(lambda_min=2.0, lambda_max=1.0) == L.OV_ERR_INVALID_ARG
    assert _create(bc_t=0) == L.OV_ERR_INVALID_ARG
    assert _create(outer_tol=-1.0) == L.OV_ERR_INVALID_ARG
    # free |H_W| in [1, 7): an interval that misses it is a spectrum error
    assert _create(lambda_min=1.5, lambda_max=8.0) == L.OV_ERR_SPECTRUM
    assert _create(lambda_min=0.01, lambda_max=5.0) == L.OV_ERR_SPECTRUM


def test_null_arguments():
    L = _lib()
    lib = L.lib()
    assert lib.ov_ctx_create(None, None, None) == L.OV_ERR_INVALID_ARG
    assert lib.ov_sign(None, None, None, 1, None) == L.OV_ERR_INVALID_ARG
    assert lib.ov_solve(None, None, None, None, 1, None) == L.OV_ERR_INVALID_ARG
    assert lib.ov_force(None, None, None, None, None, 1, None) == L.OV_ERR_INVALID_ARG
    assert lib.ov_zolotarev(0, 0.1, 1.0, None, None, None) == L.OV_ERR_INVALID_ARG
    assert lib.ov_status_string(L.OV_ERR_SPECTRUM).decode().startswith("spectrum")


def test_bench_refuses_several_gpus():
    """bench.py is a one-GPU benchmark: --gpus N > 1 exits with a message and status 2
    before touching any device."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "single-GPU" in msg["error"]


def test_traffic_record_gated_by_kernel_source():
    """The committed HBM-traffic record names the multi-shift pass code it was measured on;
    bench.py reports it only while that code, and the size of a full launch, are unchanged."""
    import importlib.util
    import json
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_ms_passes_16x4_traffic.json")))
    same = rec["kernel_source_hash"] == bench.kernel_source_hash()
    for name, fam in rec["families"].items():
        got = bench.measured_traffic(name, fam["full_launch_algorithmic_bytes"])
        assert got == ((fam["hbm_bytes_per_launch"], fam["ratio"]) if same else (None, None))
        assert bench.measured_traffic(name, fam["full_launch_algorithmic_bytes"] + 1) == (None, None)
        # the full launch of the benchmark's 16^4 system: two sources, three fields
        assert fam["full_launch_algorithmic_bytes"] == bench.full_bytes(name, 1, 16 ** 4)


@pytest.mark.parametrize("name", ["k_ms_passes_16x4_traffic.json",
                                  "k_ms_passes_16x3x32x12_traffic.json"])
def test_traffic_records_consistent(name):
    """Each committed HBM-traffic record is internally consistent: the scale factors are
    the copy calibration's bytes over its counter readings, the mean algorithmic bytes per
    launch lie within a full launch's, and the ratio is the mean HBM bytes over them."""
    import json
    rec = json.load(open(os.path.join(ROOT, "profiles", name)))
    cal = rec["calibration"]
    kib = cal["copy_bytes"] / 1024
    assert abs(cal["fetch_scale"] - kib / cal["fetch_kib"]) < 1e-3
    assert abs(cal["write_scale"] - kib / cal["write_kib"]) < 1e-3
    assert rec["families"]
    for fam in rec["families"].values():
        assert any(k.startswith("k_ms_t<") for k in fam["kernels"])
        assert any(k.startswith("k_ms_r<") for k in fam["kernels"])
        assert 0 < fam["algorithmic_bytes_per_launch"] <= fam["full_launch_algorithmic_bytes"]
        assert abs(fam["ratio"] - fam["hbm_bytes_per_launch"] / fam["algorithmic_bytes_per_launch"]) < 1e-3
        for k in fam["kernels"]:
            assert fam["dispatches"][k] > 0
            # medians of whole dispatches: written bytes never exceed a full launch's field
            field = fam["full_launch_algorithmic_bytes"] / 3
            assert fam["write_kib_median"][k] * 1024 * cal["write_scale"] <= field * 1.01


def test_record_traffic_sums_every_launch_form(tmp_path):
    """bench.py --record-traffic on a synthetic counter pair: the copy calibrates the scale
    factors, every launch form of a pass family (operands-first and check-first variants)
    is summed, each dispatch's algorithmic bytes follow from its exact writes, and the ratio
    is total HBM bytes over total algorithmic bytes."""
    import csv
    import importlib.util
    import json
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    V, systems, sources = 4096, 1, 2
    field = systems * sources * 4 * V * 8              # bytes of one FP32 output field
    fkib = field / 1024
    rows_f, rows_w = [], []
    did = 0

    def add(name, fetch_kib, write_kib):
        nonlocal did
        did += 1
        rows_f.append({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Value": fetch_kib})
        rows_w.append({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Value": write_kib})

    copy = "__amd_rocclr_copyBuffer"
    add(copy, 512 * 1024 / 2.0, 512 * 1024)            # fetch counts half the copy's bytes
    t0 = "void ov::k_ms_t<float, 2, false>(ov::SysDev const*, int const*, int, int, ov::MsParams)"
    r0 = "void ov::k_ms_r<float, 2, false>(ov::SysDev const*, int const*, int, int, ov::MsParams)"
    t1 = "void ov::k_ms_t<float, 2, true>(ov::SysDev const*, int const*, int, int, ov::MsParams)"
    add(t0, 2.0 * fkib / 2.0, fkib)                    # full launch: reads 2 fields
    add(r0, 2.6 * fkib / 2.0, fkib)                    # full launch: reads 2.6 fields
    add(t1, 1.0 * fkib / 2.0, 0.5 * fkib)              # half the entries: reads 1 field
    for path, rows in (("f.csv", rows_f), ("w.csv", rows_w)):
        with open(tmp_path / path, "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Value"])
            w.writeheader()
            w.writerows(rows)
    out = tmp_path / "rec.json"
    bench.record_traffic(str(out), str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "synthetic",
                         systems, sources, V)
    fam = json.load(open(out))["families"]["fp32_inner"]
    assert sorted(fam["kernels"]) == ["k_ms_r<float, 2, false>", "k_ms_t<float, 2, false>",
                                      "k_ms_t<float, 2, true>"]
    hbm = (2.0 + 1 + 2.6 + 1 + 1.0 + 0.5) * field      # reads + writes of the three dispatches
    alg = (3 + 3 + 1.5) * field                        # three fields per source taking part
    assert abs(fam["hbm_bytes_per_launch"] - hbm / 3) <= 1
    assert abs(fam["algorithmic_bytes_per_launch"] - alg / 3) <= 1
    assert abs(fam["ratio"] - round(hbm / alg, 3)) < 1e-9
    assert fam["full_launch_algorithmic_bytes"] == 3 * field
