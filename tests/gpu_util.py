"""Helpers shared by the GPU test modules: comparisons, host <-> device copies and the
workloads' couplings.  No arithmetic of the method lives here."""
import numpy as np

CFG1 = dict(m=0.05, g=0.1, n_poles=16, lambda_min=0.01, lambda_max=8.0)
CFG2 = dict(m=0.05, g=0.3, n_poles=20, lambda_min=1e-3, lambda_max=8.0)
CFG5 = dict(m=0.05, g=0.3, n_poles=24, lambda_min=1e-4, lambda_max=8.0)  # uneven-batch sign


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def maxabs(a, b):
    """Largest element-wise deviation, relative to the largest element of b."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.abs(a - b).max() / np.abs(b).max()


def check(a, b, tol, what=""):
    """Element by element and in norm: max |a - b| <= tol max |b| and
    ||a - b|| <= tol ||b|| (a deviation confined to a few sites fails the first)."""
    r, m = rel(a, b), maxabs(a, b)
    assert r < tol and m < tol, f"{what} rel {r:.3e} max-abs {m:.3e} (tol {tol:.1e})"
    return r, m


def require_gpu(torch):
    """Fail (not skip) without a HIP device, and load libov.so: there is no fallback."""
    import pytest
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible HIP device")
    from paper_1005_3276_amd import _lib
    _lib.lib()
    print(f"[gpu] {torch.cuda.get_device_name(0)}", flush=True)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def bits(a):
    """The bit patterns of a complex128 array (for bitwise comparisons)."""
    return np.ascontiguousarray(a).view(np.uint64)


def lattice(dims, **kw):
    from paper_1005_3276_amd import Lattice
    return Lattice(dims, **kw)
