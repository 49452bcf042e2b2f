"""Benchmark: overlap solves/s at 16^4 (mixed FP32/FP64 vs FP64) to a 1e-10
true residual, plus the Wilson-stencil bandwidth.

One step = one solve of M^dag M x = b at 16^4 (m = 0.05, g = 0.3, phi ~ CN(0, 0.25),
20 Zolotarev poles on [1e-3, 8], outer residual 1e-10) with the mixed-precision
solver: every step of the hot path (pack, multi-shift sign, D_ov / M / M^dag
epilogues, free-field preconditioner, outer CG, reliable FP64 updates) runs
inside it.  Inputs are seeded synthetic fields resident in HBM before the timed
region.

Prints ONE JSON line.  Only one GPU is supported: --gpus N > 1 exits.
"""
import argparse
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DIMS = (16, 16, 16, 16)
CFG = dict(m=0.05, g=0.3, n_poles=20, lambda_min=1e-3, lambda_max=8.0, outer_tol=1e-10,
           inner_tol=1e-8, truth_tol=1e-13)
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the multi-shift pass code (ov_common.hpp + ZmMarch .. ms_r_block)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1005_3276_amd", "csrc")
    common = open(os.path.join(csrc, "ov_common.hpp")).read()
    kern = open(os.path.join(csrc, "ov_kernels.hpp")).read()
    a = kern.index("struct ZmMarch {")
    b = kern.index("// Iteration n, t pass:")
    return hashlib.sha256((common + kern[a:b]).encode()).hexdigest()[:16]


TRAFFIC_RECORDS = ("k_ms_passes_16x4_traffic.json", "k_ms_passes_16x3x32x12_traffic.json")


def measured_traffic(family, full_launch_bytes):
    """Mean HBM bytes per launch of a pass family and their ratio to the mean algorithmic
    bytes, from the committed counter runs (one record per workload, told apart by the
    algorithmic bytes of a full launch), if the kernels are unchanged; else (None, None)."""
    for name in TRAFFIC_RECORDS:
        try:
            rec = json.load(open(os.path.join(ROOT, "profiles", name)))
        except (OSError, ValueError):
            continue
        if rec.get("kernel_source_hash") != kernel_source_hash():
            continue
        f = rec.get("families", {}).get(family)
        if f and abs(f.get("full_launch_algorithmic_bytes", -1) - full_launch_bytes) <= 0.5:
            return f.get("hbm_bytes_per_launch"), f.get("ratio")
    return None, None


def stencil_bandwidth(lat, torch, nrhs, prec, reps=20):
    """Algorithmic bytes (read + write one spinor per site) / kernel time."""
    V = lat.V
    dt = torch.complex64 if prec else torch.complex128
    x = torch.randn((nrhs, 4, V), dtype=dt, device="cuda")
    lat.stencil_bench(x, prec, reps=2)
    _, ms = lat.stencil_bench(x, prec, reps=reps)
    esize = 8 if prec else 16
    gbs = 2.0 * 4 * esize * V * nrhs / (ms * 1e-3) / 1e9
    return {"nrhs": nrhs, "prec": "fp32" if prec else "fp64", "ms": ms, "GB_s": gbs,
            "frac_hbm": gbs / HBM_PEAK_GBS}


def stencil_sweep(lat, torch):
    """H_W alone at 16^4: 1, 12, 48 right-hand sides in FP32 and FP64, then beyond the
    256 MB Infinity Cache (192 FP32 / 96 FP64 fields)."""
    sweep = []
    for prec in (1, 0):
        for nrhs in (1, 12, 48):
            sweep.append(stencil_bandwidth(lat, torch, nrhs, prec))
            log(f"stencil {sweep[-1]}")
    for nrhs, prec in ((192, 1), (96, 0)):
        sweep.append(stencil_bandwidth(lat, torch, nrhs, prec))
        log(f"stencil {sweep[-1]}")
    return sweep


def record_traffic(out_path, fetch_csv, write_csv, workload, systems, sources, volume):
    """Host only: the HBM traffic record of the multi-shift pass families from two rocprofv3
    --pmc runs of one command (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), scaled by the
    largest device copy in the same program (run with --calibrate-copy: 512 MiB each way).
    The two runs dispatch the same deterministic sequence, so the n-th dispatch of a kernel
    in one is the n-th in the other.  Writes are exact (one output field per source taking
    part), so each dispatch's WRITE_SIZE gives the share of the launch's systems that took
    part, and with it the dispatch's algorithmic bytes (3 fields per source).  Records the
    mean HBM bytes per launch against the mean algorithmic bytes per launch and their ratio
    (sums over every dispatch), the full launch's algorithmic bytes (every system and source
    taking part: the key bench.py matches on) and the per-kernel medians.  Writes the JSON
    that measured_traffic reads."""
    import csv
    import statistics

    def per_kernel(path):
        by = {}
        for r in csv.DictReader(open(path)):
            by.setdefault(r["Kernel_Name"], []).append(
                (int(r["Dispatch_Id"]), float(r["Counter_Value"])))
        return {k: [v for _, v in sorted(x)] for k, x in by.items()}

    fetch, write = per_kernel(fetch_csv), per_kernel(write_csv)
    copy = [k for k in fetch if "copyBuffer" in k]
    cf = max(max(fetch[k]) for k in copy)
    cw = max(max(write[k]) for k in copy)
    copy_kib = 512 * 1024
    fs, ws = copy_kib / cf, copy_kib / cw
    rec = {"kernel_source_hash": kernel_source_hash(),
           "hash_covers": "ov_common.hpp + ov_kernels.hpp from struct ZmMarch to the k_ms_t comment",
           "workload": workload,
           "calibration": {"copy_bytes": copy_kib * 1024, "fetch_kib": cf, "write_kib": cw,
                           "fetch_scale": fs, "write_scale": ws},
           "families": {}}
    for fam, prec, esize in (("fp32_inner", "float", 8), ("fp64_truth", "double", 16)):
        # every launch form of the family's two passes (plain / z-marching variants)
        full = {}
        for n in fetch:
            m = re.search(r"(k_ms_[tr]<%s, [^>]*>)" % prec, n)
            if m and n in write:
                full[m.group(1)] = n
        ks = sorted(full)
        if not any(k.startswith("k_ms_t") for k in ks) or not any(k.startswith("k_ms_r") for k in ks):
            continue
        field = systems * sources * 4 * volume * esize  # one field per source, whole launch
        alg_full = 3 * field
        hbm, alg, n = 0.0, 0.0, 0
        for k in ks:
            for f_kib, w_kib in zip(fetch[full[k]], write[full[k]]):
                hbm += (f_kib * fs + w_kib * ws) * 1024
                alg += alg_full * min(1.0, w_kib * ws * 1024 / field)
                n += 1
        rec["families"][fam] = {
            "kernels": ks, "sources_per_launch": sources * systems,
            "fetch_kib_median": {k: statistics.median(fetch[full[k]]) for k in ks},
            "write_kib_median": {k: statistics.median(write[full[k]]) for k in ks},
            "dispatches": {k: min(len(fetch[full[k]]), len(write[full[k]])) for k in ks},
            "hbm_bytes_per_launch": round(hbm / n),
            "algorithmic_bytes_per_launch": round(alg / n),
            "full_launch_algorithmic_bytes": alg_full,
            "ratio": round(hbm / alg, 3)}
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=2)
    print(json.dumps(rec["families"], indent=1))


def calibrate_copy(torch):
    """One 512 MiB device copy: the reference dispatch for the traffic counters."""
    nbytes = 512 << 20
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()


def copy_bandwidth(torch):
    """Read + write bandwidth of a plain device copy (torch) at the stencil's working
    set sizes: the streaming bandwidth this part reaches in practice."""
    out = {}
    for mib in (100, 800):
        n = mib << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        out[f"{mib}MiB"] = 2.0 * n / (ms * 1e-3) / 1e12
        del a, b
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def oracle_solve_timed(dims, phi, b, m=0.05, g=0.3, inner_tol=1e-12):
    """One complete solve of MdagM x = b by the FP64 oracle (its plain CG on MdagM,
    multi-shift tolerance inner_tol, stop on the true residual 1e-10), timed."""
    from oracle import oracle as O
    o = O.Oracle(dims, m=m, g=g, n_poles=CFG["n_poles"], lambda_min=CFG["lambda_min"],
                 lambda_max=CFG["lambda_max"], inner_tol=inner_tol)
    t = time.perf_counter()
    _, st, rc = o.solve(b, phi, tol=CFG["outer_tol"], maxit=2000)
    el = time.perf_counter() - t
    return el, {"seconds": el, "outer_iters": st.iters, "inner_iters": st.inner_iters,
                "true_rel_res": st.true_rel_res, "converged": rc == 0}


def cpu_baseline(phi, src):
    """The oracle on the host cores: one complete solve of the benchmark's own system
    (16^4, same inputs), timed whole."""
    from oracle import oracle as O
    el, st = oracle_solve_timed(DIMS, phi, src[0])
    return {"value": 1.0 / el, "unit": "solves/s", "cores": O.threads(), "kind": "oracle",
            "cpu": cpu_model(), "timed": "complete solve",
            "sample": f"one complete solve of the benchmark's system at 16^4 by the FP64 oracle "
                      f"(plain CG on MdagM, no preconditioner, multi-shift tol 1e-12): "
                      f"{st['outer_iters']} CG iterations, true residual "
                      f"{st['true_rel_res']:.2e}, {el:.1f} s",
            "solve": st}


def cpu_suite(full16):
    """--cpu-only: the oracle timed on the config-2 solves (8^4, and 16^4 with full16)
    and the config-4 force (12^4), with the threads OMP_NUM_THREADS gives it."""
    from oracle import oracle as O
    from paper_1005_3276_amd import inputs
    out = {"metric": "cpu_oracle", "cores": O.threads(), "cpu": cpu_model()}
    phi, src = inputs.draw((8, 8, 8, 8), nrhs=1, sigma2=0.25, seed=inputs.config_seed(2) + 1)
    out["solve_8x4"] = oracle_solve_timed((8, 8, 8, 8), phi, src[0])[1]
    log(f"oracle 8^4 solve: {out['solve_8x4']}")
    if full16:
        phi, src = inputs.draw(DIMS, nrhs=1, sigma2=0.25, seed=inputs.config_seed(2))
        out["solve_16x4"] = oracle_solve_timed(DIMS, phi, src[0])[1]
        log(f"oracle 16^4 solve: {out['solve_16x4']}")
    d12 = (12, 12, 12, 12)
    phi, xi = inputs.draw(d12, nrhs=1, sigma2=0.25, seed=inputs.config_seed(4))
    o = O.Oracle(d12, m=0.05, g=0.3, n_poles=20, lambda_min=1e-3, lambda_max=8.0,
                 inner_tol=1e-12)
    t = time.perf_counter()
    S, _, st, rc = o.force(phi, xi[0], tol=CFG["outer_tol"])
    el = time.perf_counter() - t
    out["force_12x4"] = {"seconds": el, "S": S, "outer_iters": st.iters,
                         "true_rel_res": st.true_rel_res, "converged": rc == 0}
    log(f"oracle 12^4 force: {out['force_12x4']}")
    return out


def full_bytes(family, systems, volume):
    """Algorithmic bytes of one multi-shift pass launch with every system taking part: two
    sources per system (the Ginsparg-Wilson forms), three fields each (two read, one
    written), 4 spins of 8 B (FP32) or 16 B (FP64) per site."""
    esize = 8 if family == "fp32_inner" else 16
    return 3 * 2 * systems * 4 * volume * esize


# multi-shift pass families: (t-pass kernel id, r-pass kernel id) of the library's
# event sampling (ov_kernel_sampling): 0/1 FP32 passes, 3/4 FP64 passes
FAMILIES = {"fp64_truth": (3, 4), "fp32_inner": (0, 1)}


def sampled_spans(lat, run):
    """Run `run()` once with every multi-shift pass launch sampled by HIP events on the
    library's stream (and device wall-clock stamps of every workgroup)."""
    lat.kernel_sampling(512)
    for k in range(5):
        lat.kernel_spans(k, reset=True)
    run()
    lat.kernel_sampling(0)
    return [lat.kernel_spans(k) for k in range(5)]  # (kernel_ms, kcnt, event_ms, cnt, bytes)


def family_roofline(spans, name, kname, full_launch_bytes):
    """Achieved algorithmic GB/s of one pass family over the sampled launches.  The bytes
    of a launch are those of the systems that took part (the library counts the sites its
    workgroups processed); full_launch_bytes is a launch with every system taking part."""
    ids = FAMILIES[name]
    ms_sum = sum(spans[k][2] for k in ids)
    cnt = sum(spans[k][3] for k in ids)
    bytes_sum = sum(spans[k][4] for k in ids)
    per_launch = bytes_sum / max(cnt, 1)
    achieved = bytes_sum / (ms_sum * 1e-3) / 1e9 if ms_sum > 0 else 0.0
    traffic, ratio = measured_traffic(name, full_launch_bytes)
    r = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_ratio": ratio,
         "kernel": kname, "avg_launch_us": ms_sum / max(cnt, 1) * 1e3,
         "bytes_per_launch": per_launch, "full_launch_bytes": full_launch_bytes,
         "active_share": per_launch / full_launch_bytes, "launches_per_solve": cnt,
         "event_ms_per_solve": ms_sum,
         "t_pass_us": spans[ids[0]][2] / max(spans[ids[0]][3], 1) * 1e3,
         "r_pass_us": spans[ids[1]][2] / max(spans[ids[1]][3], 1) * 1e3}
    # the same launches, kernel-only: max(end) - min(start) of device wall-clock
    # stamps taken by every workgroup (what a kernel trace reports; the event
    # duration above also holds the dispatch gap before each launch)
    kms = sum(spans[k][0] for k in ids)
    kcnt = sum(spans[k][1] for k in ids)
    if kcnt > 0:
        r["kernel_only_us"] = kms / kcnt * 1e3
        r["achieved_kernel_only"] = per_launch / (kms / kcnt * 1e-3) / 1e9
    return r


def batched_config3(torch, Lattice, inputs):
    """The batched workload (12 sources on 16^3 x 32, mixed): timed solve, then one
    sampled solve giving the pass families' achieved bandwidth at that size."""
    dims = (16, 16, 16, 32)
    phi, src = inputs.draw(dims, nrhs=12, sigma2=0.5, seed=inputs.config_seed(3))
    lat = Lattice(dims, precision="mixed", m=0.02, g=0.5, n_poles=20, lambda_min=1e-3,
                  lambda_max=8.0, outer_tol=1e-10)
    b, p = torch.from_numpy(src).cuda(), torch.from_numpy(phi).cuda()
    lat.solve(b, p)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, st = lat.solve(b, p)
    torch.cuda.synchronize()
    e = time.perf_counter() - t
    spans = sampled_spans(lat, lambda: lat.solve(b, p))
    out = {"seconds": e, "rhs_solves_per_s": 12 / e,
           "max_true_rel_res": max(s["true_rel_res"] for s in st),
           "outer_iters": [s["outer_iters"] for s in st],
           "pass_rooflines": {
               n: family_roofline(spans, n, k, full_bytes(n, 12, 16 * 16 * 16 * 32)) for n, k in (
                   ("fp32_inner", "k_ms_t<float, *> + k_ms_r<float, *> (FP32 inner passes, "
                                  "12 systems x 2 sources per launch)"),
                   ("fp64_truth", "k_ms_t<double, *> + k_ms_r<double, *> (FP64 true-residual "
                                  "passes, the systems due for an update x 2 sources per launch)"))}}
    del lat
    return out, b, p


def other_configs(torch, Lattice, inputs):
    """Timed runs of the batched (16^3x32, 12 rhs), force (12^4) and uneven-batch
    workloads; one warm-up and one timed call each."""
    from paper_1005_3276_amd import solve_batch
    out = {}
    # config 3
    dims = (16, 16, 16, 32)
    c3, b, p = batched_config3(torch, Lattice, inputs)
    e = c3["seconds"]
    out["config3_batched_16x3x32_12rhs"] = c3
    log(f"config3: {out['config3_batched_16x3x32_12rhs']}")
    # the same batch with the FP64 solver (the mixed solver's algorithm in FP64)
    lat = Lattice(dims, precision="fp64", m=0.02, g=0.5, n_poles=20, lambda_min=1e-3,
                  lambda_max=8.0, outer_tol=1e-10, inner_tol=1e-8)
    lat.solve(b, p)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, st = lat.solve(b, p)
    torch.cuda.synchronize()
    e64 = time.perf_counter() - t
    out["config3_batched_16x3x32_12rhs_fp64"] = {
        "seconds": e64, "rhs_solves_per_s": 12 / e64,
        "max_true_rel_res": max(s["true_rel_res"] for s in st),
        "mixed_speedup": e64 / e}
    log(f"config3 fp64: {out['config3_batched_16x3x32_12rhs_fp64']}")
    del lat
    # config 4
    dims = (12, 12, 12, 12)
    phi, xi = inputs.draw(dims, nrhs=1, sigma2=0.25, seed=inputs.config_seed(4))
    lat = Lattice(dims, precision="mixed", m=0.05, g=0.3, n_poles=20, lambda_min=1e-3,
                  lambda_max=8.0, outer_tol=1e-10)
    x_, p_ = torch.from_numpy(xi).cuda(), torch.from_numpy(phi).cuda()
    lat.force(x_, p_)
    torch.cuda.synchronize()
    t = time.perf_counter()
    S, G, st = lat.force(x_, p_)
    torch.cuda.synchronize()
    e = time.perf_counter() - t
    out["config4_force_12x4"] = {"seconds": e, "forces_per_s": 1 / e, "S": S[0],
                                 "outer_iters": st[0]["outer_iters"]}
    log(f"config4: {out['config4_force_12x4']}")
    del lat
    # config 5
    members = [((8, 8, 8, 8), 4), ((12, 12, 12, 12), 4), ((16, 16, 16, 16), 2),
               ((24, 24, 24, 48), 1)]
    lats, bs, ps = [], [], []
    for k, (d, n) in enumerate(members):
        phi, src = inputs.draw(d, nrhs=n, sigma2=0.25, seed=inputs.config_seed(5) + k)
        lats.append(Lattice(d, precision="mixed", m=0.05, g=0.3, n_poles=24, lambda_min=1e-4,
                            lambda_max=8.0, outer_tol=1e-10))
        bs.append(torch.from_numpy(src).cuda())
        ps.append(torch.from_numpy(phi).cuda())
    solve_batch(lats, bs, ps)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, st = solve_batch(lats, bs, ps)
    torch.cuda.synchronize()
    e = time.perf_counter() - t
    out["config5_uneven_batch"] = {
        "seconds": e, "rhs_solves_per_s": 11 / e,
        "max_true_rel_res": max(s["true_rel_res"] for s in st),
        "outer_iters": [s["outer_iters"] for s in st]}
    log(f"config5: {out['config5_uneven_batch']}")
    # the adjoint force on the 16^4 member (its first source)
    l16 = lats[2]
    xi16 = bs[2][:1].contiguous()
    l16.force(xi16, ps[2])
    torch.cuda.synchronize()
    t = time.perf_counter()
    S16, _, st16 = l16.force(xi16, ps[2])
    torch.cuda.synchronize()
    e16 = time.perf_counter() - t
    out["config5_force_16x4_member"] = {"seconds": e16, "S": S16[0],
                                        "outer_iters": st16[0]["outer_iters"]}
    log(f"config5 force: {out['config5_force_16x4_member']}")
    del lats
    # the same batch with the FP64 solver
    lats = [Lattice(d, precision="fp64", m=0.05, g=0.3, n_poles=24, lambda_min=1e-4,
                    lambda_max=8.0, outer_tol=1e-10, inner_tol=1e-8) for d, _ in members]
    solve_batch(lats, bs, ps)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, st = solve_batch(lats, bs, ps)
    torch.cuda.synchronize()
    e64 = time.perf_counter() - t
    out["config5_uneven_batch_fp64"] = {
        "seconds": e64, "rhs_solves_per_s": 11 / e64,
        "max_true_rel_res": max(s["true_rel_res"] for s in st),
        "mixed_speedup": e64 / e}
    log(f"config5 fp64: {out['config5_uneven_batch_fp64']}")
    return out


def momentum_forms(torch, Lattice, inputs, dphi, dsrc):
    """The paper's own operator route (Sec. 7.2-7.3): the Dirac operator applied
    exactly in momentum space (exact-sign D_ov, and the paper's Dslash), with and
    without the free-field preconditioner; at 16^4 with the workload's couplings
    and at 16^3 x 32 with the m = 1, g = 1/5 of the paper's inversion benchmarks."""
    out = {}

    def timed(lat, b, p):
        lat.solve(b, p)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = lat.solve(b, p)
        torch.cuda.synchronize()
        return time.perf_counter() - t, st[0]

    # unpreconditioned Dslash at m = 0.05 needs thousands of iterations
    cfg = dict(CFG, max_outer=20000)
    for dirac in ("overlap_exact", "dslash"):
        for prec in ("mixed", "fp64"):
            for pc in (1, 0):
                lat = Lattice(DIMS, precision=prec, dirac=dirac, precondition=pc, **cfg)
                e, st = timed(lat, dsrc, dphi)
                out[f"fft_{dirac}_{prec}_pc{pc}_16x4"] = {
                    "ms_per_solve": e * 1e3, "solves_per_s": 1 / e,
                    "outer_iters": st["outer_iters"], "true_rel_res": st["true_rel_res"]}
                log(f"{dirac} {prec} pc={pc} 16^4: {out[f'fft_{dirac}_{prec}_pc{pc}_16x4']}")
                del lat
    dims = (16, 16, 16, 32)
    phi, src = inputs.draw(dims, nrhs=1, sigma2=0.25, seed=inputs.config_seed(2))
    b, p = torch.from_numpy(src).cuda(), torch.from_numpy(phi).cuda()
    for prec in ("mixed", "fp64"):
        for pc in (1, 0):
            lat = Lattice(dims, precision=prec, dirac="dslash", precondition=pc, m=1.0, g=0.2,
                          outer_tol=1e-10, max_outer=20000)
            e, st = timed(lat, b, p)
            out[f"fft_dslash_{prec}_pc{pc}_16x3x32_m1_g0.2"] = {
                "ms_per_solve": e * 1e3, "outer_iters": st["outer_iters"],
                "true_rel_res": st["true_rel_res"]}
            log(f"dslash 16^3x32 {prec} pc={pc}: {out[f'fft_dslash_{prec}_pc{pc}_16x3x32_m1_g0.2']}")
            del lat
    # RHMC rational layers (Sec. 7.3): heatbath (MdagM)^{1/8} R then the action's
    # (MdagM)^{-1/4}, degree 20 on [1e-5, 10], with the multi-shift D_ov of the workload
    from paper_1005_3276_amd import rational
    c18 = rational.power_approx(0.125, 1e-5, 10.0, 20)
    c14 = rational.power_approx(-0.25, 1e-5, 10.0, 20)
    for dirac in ("overlap_exact", "overlap"):
        lat = Lattice(DIMS, dirac=dirac, inner_tol=1e-12, outer_tol=1e-10,
                      **{k: v for k, v in CFG.items() if k not in ("outer_tol", "inner_tol")})
        lat.rational(dsrc, dphi, *c18[:3])
        torch.cuda.synchronize()
        t = time.perf_counter()
        eta, st1 = lat.rational(dsrc, dphi, *c18[:3])
        w, st2 = lat.rational(eta, dphi, *c14[:3])
        torch.cuda.synchronize()
        e = time.perf_counter() - t
        lhs = torch.vdot(eta.reshape(-1), w.reshape(-1)).real.item()
        rhs = torch.vdot(dsrc.reshape(-1), dsrc.reshape(-1)).real.item()
        out[f"rhmc_heatbath_action_{dirac}_16x4"] = {
            "seconds": e, "iterations": [st1[0]["outer_iters"], st2[0]["outer_iters"]],
            "identity_rel_dev": abs(lhs - rhs) / rhs,
            "fit_rel_err": [c18[3], c14[3]]}
        log(f"rhmc {dirac}: {out[f'rhmc_heatbath_action_{dirac}_16x4']}")
        del lat
    # the paper's heatbath workload (Sec. 7.3, Table heattab1, context only): eta =
    # (MdagM)^{1/8} R with the Dslash fermion matrix at m = 1, g = 0.1, degree 20 on the
    # free spectrum of M0^dag M0 ([1.01, 8.2e4] on these lattices: fit on [1, 1e5]); shifts
    # beta_i <= 100 by the preconditioned solver (the paper's cutoff), the rest by one
    # multi-shift CG; iterations summed over the 20 shifts, as the table counts them
    c18p = rational.power_approx(0.125, 1.0, 1e5, 20)
    for dims in ((8, 8, 8, 32), (16, 16, 16, 32)):
        phi, src = inputs.draw(dims, nrhs=1, sigma2=0.25, seed=inputs.config_seed(2) + 7)
        b, p = torch.from_numpy(src).cuda(), torch.from_numpy(phi).cuda()
        tag = "x".join(str(d) for d in dims)
        for prec in ("mixed", "fp64"):
            for cut in (100.0, 0.0):
                lat = Lattice(dims, precision=prec, dirac="dslash", m=1.0, g=0.1, outer_tol=1e-10,
                              shift_pc_cutoff=cut)
                lat.rational(b, p, *c18p[:3])
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, st = lat.rational(b, p, *c18p[:3])
                torch.cuda.synchronize()
                e = time.perf_counter() - t
                key = f"heatbath_dslash_{prec}_{'pc100' if cut else 'multishift'}_{tag}_m1_g0.1"
                out[key] = {"seconds": e, "iterations_summed": st[0]["outer_iters"],
                            "fit_rel_err": c18p[3]}
                log(f"heatbath {tag} {prec} cutoff {cut}: {out[key]}")
                del lat
    # locality probe of Dslash on 16^4 (Sec. 3.2, Fig. rfig)
    lat = Lattice(DIMS, dirac="dslash")
    lat.locality(0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    f, _ = lat.locality(0)
    e = time.perf_counter() - t
    out["locality_dslash_16x4"] = {"seconds": e, "f": [float(v) for v in f]}
    log(f"locality: {e * 1e3:.2f} ms")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip FP64, stencil and other configs")
    ap.add_argument("--no-sample", action="store_true", help="skip the event-sampled solve")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shape (256 threads, 1 site per thread at 16^4)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with one 512 MiB device copy (reference for traffic counters)")
    ap.add_argument("--stencil-only", action="store_true",
                    help="only the 16^4 stencil sweep (one JSON line of its own)")
    ap.add_argument("--cpu-only", action="store_true",
                    help="only the oracle timings on the host (config-2 solve at 8^4, config-4 "
                         "force at 12^4; no GPU); one JSON line")
    ap.add_argument("--cpu-16", action="store_true",
                    help="with --cpu-only: also the config-2 solve at 16^4")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched 12 x 16^3x32 mixed solve with its pass rooflines "
                         "(one JSON line of its own)")
    ap.add_argument("--record-traffic", nargs=7,
                    metavar=("OUT_JSON", "FETCH_CSV", "WRITE_CSV", "WORKLOAD", "SYSTEMS",
                             "SOURCES", "VOLUME"),
                    help="host only: write the pass families' traffic record from two "
                         "rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE)")
    args = ap.parse_args()
    if args.record_traffic:
        o, fc, wc, wl, nsys, nsrc, vol = args.record_traffic
        record_traffic(o, fc, wc, wl, int(nsys), int(nsrc), int(vol))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU benchmark: run with --gpus 1 (the batched "
                                   "and multi-lattice work would shard across GPUs without "
                                   "communication; no multi-GPU path is implemented)"}))
        sys.exit(2)

    if args.cpu_only:
        print(json.dumps(cpu_suite(args.cpu_16)), flush=True)
        return

    import numpy as np
    import torch

    from paper_1005_3276_amd import Lattice, inputs

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.stencil_only:
        lat = Lattice(DIMS, **CFG)
        stencil_bandwidth(lat, torch, 48, 1, reps=20)  # clocks up
        sweep = stencil_sweep(lat, torch)
        out = {"metric": "stencil_only", "stencil": sweep,
               "stencil_best_TB_s": max(s["GB_s"] for s in sweep) / 1e3}
        if args.calibrate_copy:
            calibrate_copy(torch)
            out["calibration_copy_bytes"] = 512 << 20
        print(json.dumps(out), flush=True)
        return
    if args.batched_only:
        c3, _, _ = batched_config3(torch, Lattice, inputs)
        out = {"metric": "batched_only", "config3_batched_16x3x32_12rhs": c3}
        if args.calibrate_copy:
            calibrate_copy(torch)
            out["calibration_copy_bytes"] = 512 << 20
        print(json.dumps(out), flush=True)
        return
    phi, src = inputs.draw(DIMS, nrhs=1, sigma2=0.25, seed=inputs.config_seed(2))
    dphi = torch.from_numpy(phi).cuda()
    dsrc = torch.from_numpy(src).cuda()
    lat = Lattice(DIMS, precision="mixed", **CFG)
    lat.use_workspace(1)
    from paper_1005_3276_amd import tune
    if args.no_tune:
        choice, tune_us = None, None
    else:
        # candidates timed on the benchmark's own step (one solve)
        choice, tune_us = tune.autotune(lat, prec=1, nrhs=1, workload=lambda: lat.solve(dsrc, dphi),
                                        tag="solve")
    log(f"autotune: {choice} {tune_us}")

    # ---- mixed solves (the metric)
    for _ in range(args.warmup):
        lat.solve(dsrc, dphi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for _ in range(args.steps):
        x, stats = lat.solve(dsrc, dphi)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = args.steps / el
    log(f"mixed: {el / args.steps * 1e3:.2f} ms/solve  {stats[0]}")

    # ---- dominant kernel: live HIP-event sampling on the library's stream.  Every
    # multi-shift pass launch of one solve is sampled (the cap applies per host
    # synchronisation, i.e. per outer iteration / reliable update), so the per-family
    # sums below cover the whole solve and decide which pass family dominates.
    families = {
        "fp64_truth": "k_ms_t<double, *> + k_ms_r<double, *> (FP64 multi-shift passes of "
                      "the true residuals, two sources per launch)",
        "fp32_inner": "k_ms_t<float, *> + k_ms_r<float, *> (FP32 multi-shift passes of "
                      "the inner CG, two sources per launch)",
    }
    if args.no_sample:
        lat.kernel_sampling(0)
        for k in range(5):
            lat.kernel_spans(k, reset=True)
        lat.solve(dsrc, dphi)
        spans = [lat.kernel_spans(k) for k in range(5)]
    else:
        spans = sampled_spans(lat, lambda: lat.solve(dsrc, dphi))

    fam = {n: family_roofline(spans, n, families[n], full_bytes(n, 1, lat.V)) for n in families}
    dom = max(fam, key=lambda n: fam[n]["event_ms_per_solve"])
    roofline = fam[dom]
    roofline_secondary = fam[[n for n in fam if n != dom][0]]
    log(f"roofline: {roofline}")

    extra = {}
    if not args.quick:
        # ---- plain FP64 paths (P2: inner 1e-8 + reliable updates; P1: inner 1e-12)
        # P1: plain nested FP64 CG, inner sign at 1e-12, no reliable updates
        # P2: FP64 with reliable updates, inner sign fixed at 1e-8
        # P3: FP64 running the mixed solver's algorithm (relaxed inner sign)
        # (all preconditioned like the mixed solve; *_unpreconditioned without it)
        for name, kw in (("fp64_p1", dict(inner_tol=1e-12, reliable_delta=0.0, inner_relax=0.0)),
                         ("fp64_p2", dict(inner_tol=1e-8, reliable_delta=0.1, inner_relax=0.0)),
                         ("fp64_p3", dict(inner_tol=1e-8)),
                         # without the preconditioner CG on MdagM converges unevenly and
                         # long FP32 cycles lose accuracy: reliable updates every 100x
                         ("fp64_p3_unpreconditioned", dict(inner_tol=1e-8, precondition=0,
                                                           reliable_delta=0.01, inner_relax=1e-3)),
                         ("mixed_unpreconditioned", dict(precision="mixed", precondition=0,
                                                         reliable_delta=0.01, inner_relax=1e-3))):
            cfg = dict(CFG, precision="fp64")
            cfg.update(kw)
            l64 = Lattice(DIMS, **cfg)
            l64.solve(dsrc, dphi)
            torch.cuda.synchronize()
            t = time.perf_counter()
            x64, st64 = l64.solve(dsrc, dphi)
            torch.cuda.synchronize()
            e64 = time.perf_counter() - t
            extra[name] = {"solves_per_s": 1.0 / e64, "ms_per_solve": e64 * 1e3,
                           "outer_iters": st64[0]["outer_iters"],
                           "inner_iters": st64[0]["inner_iters"],
                           "true_rel_res": st64[0]["true_rel_res"]}
            log(f"{name}: {extra[name]}")
            del l64
        best64 = max(extra[k]["solves_per_s"] for k in ("fp64_p1", "fp64_p2", "fp64_p3"))
        extra["mixed_speedup_vs_best_fp64"] = value / best64
        # ---- the same workload at 8^4 (the smaller lattice of the workload), mixed vs FP64
        d8 = (8, 8, 8, 8)
        phi8, src8 = inputs.draw(d8, nrhs=1, sigma2=0.25, seed=inputs.config_seed(2) + 1)
        b8, p8 = torch.from_numpy(src8).cuda(), torch.from_numpy(phi8).cuda()
        r8 = {}
        for name, kw in (("mixed", dict(precision="mixed")),
                         ("fp64_p3", dict(precision="fp64", inner_tol=1e-8))):
            l8 = Lattice(d8, **dict(CFG, **kw))
            l8.solve(b8, p8)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(3):
                _, st8 = l8.solve(b8, p8)
            torch.cuda.synchronize()
            e8 = (time.perf_counter() - t) / 3
            r8[name] = {"ms_per_solve": e8 * 1e3, "outer_iters": st8[0]["outer_iters"],
                        "true_rel_res": st8[0]["true_rel_res"]}
            del l8
        r8["mixed_speedup"] = r8["fp64_p3"]["ms_per_solve"] / r8["mixed"]["ms_per_solve"]
        extra["config2_8x4"] = r8
        log(f"config2 8^4: {r8}")
        # ---- stencil bandwidth at 16^4
        sweep = stencil_sweep(lat, torch)
        extra["stencil"] = sweep
        extra["stencil_best_TB_s"] = max(s["GB_s"] for s in sweep) / 1e3
        extra["device_copy_TB_s"] = copy_bandwidth(torch)
        log(f"device copy: {extra['device_copy_TB_s']}")

    if not args.quick:
        extra.update(other_configs(torch, Lattice, inputs))
        extra.update(momentum_forms(torch, Lattice, inputs, dphi, dsrc))

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(phi, src)
        log(f"cpu: {cpu}")

    out = {
        "metric": "overlap solves/sec + stencil HBM TB/s at 16^4, FP32-mixed vs FP64, 1e-10 res",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "MdagM x = b at 16^4 (config 2): M = D_ov + Yukawa, m=0.05, "
                               "g=0.3, phi~CN(0,0.25), 20-pole Zolotarev on [1e-3,8], "
                               "one Gaussian rhs, true residual 1e-10, mixed FP32/FP64",
                   "lattice": list(DIMS), "nrhs": 1,
                   "true_rel_res": stats[0]["true_rel_res"],
                   "outer_iters": stats[0]["outer_iters"],
                   "inner_iters": stats[0]["inner_iters"]},
        "roofline": roofline,
        "roofline_secondary": roofline_secondary,
        "cpu_baseline": cpu,
        "autotune": {"block_x_sites_per_thread": list(choice) if choice else None,
                     "us_per_solve": tune_us},
    }
    out.update(extra)
    if args.calibrate_copy:
        calibrate_copy(torch)
        out["calibration_copy_bytes"] = 512 << 20
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
