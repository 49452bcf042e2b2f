"""Autotuner of the launch shape (threads per workgroup, sites per thread).

The native probe ``ov_tune_ms`` times the solver's hot loop (multi-shift t and
r passes) for one candidate; this driver sweeps the candidates, applies the
fastest with ``ov_set_launch`` and remembers it in a JSON cache keyed by
(device architecture, lattice, precision, right-hand sides).  Every candidate
computes the same result up to the summation order of the reductions.

Environment: OV_TUNE=0 disables tuning (keep defaults), OV_TUNE=force re-tunes
even when cached; OV_TUNE_CACHE sets the cache path
(default ~/.cache/ovwz/tune.json).
"""
import ctypes as C
import json
import os

from . import _lib as L

CANDIDATES = [(b, s) for b in (64, 128, 256) for s in (1, 2, 4)]


def _cache_path():
    return os.environ.get("OV_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ovwz", "tune.json"))


def _arch():
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName
    except Exception:
        return "unknown"


def probe(lattice, prec, nrhs, block, spt, iters=24):
    us = C.c_float()
    L.check(L.lib().ov_tune_ms(lattice._h, prec, nrhs, block, spt, iters, C.byref(us)),
            lattice._h)
    return us.value


def _time_workload(workload, reps=2):
    import time
    import torch
    workload()  # warm (graphs, iteration estimates)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t = time.perf_counter()
        workload()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best * 1e6


def autotune(lattice, prec=1, nrhs=1, iters=24, candidates=CANDIDATES, workload=None, tag=""):
    """Pick (block, sites_per_thread) for this lattice; returns (choice, timings in us).

    Without ``workload`` each candidate is timed on ``iters`` multi-shift iterations
    (``ov_tune_ms``); with it (a callable running the real work on this lattice, e.g.
    one solve) on that work itself, and ``tag`` names it in the cache key.
    """
    mode = os.environ.get("OV_TUNE", "1")
    if mode == "0":
        return None, {}
    key = f"{_arch()}|{'x'.join(map(str, lattice.dims))}|{'fp32' if prec else 'fp64'}|{nrhs}"
    if workload is not None:
        key += f"|{tag or 'workload'}"
    path = _cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache and mode != "force":
        b, s = cache[key]["block"], cache[key]["sites_per_thread"]
        lattice.set_launch(b, s)
        return (b, s), cache[key].get("us", {})
    timings = {}
    for b, s in candidates:
        if workload is not None:
            lattice.set_launch(b, s)
            timings[f"{b}x{s}"] = _time_workload(workload)
        else:
            probe(lattice, prec, nrhs, b, s, iters=4)  # warm the code path
            timings[f"{b}x{s}"] = probe(lattice, prec, nrhs, b, s, iters=iters)
    best = min(timings, key=timings.get)
    b, s = (int(v) for v in best.split("x"))
    lattice.set_launch(b, s)
    cache[key] = {"block": b, "sites_per_thread": s, "us": timings}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass
    return (b, s), timings
