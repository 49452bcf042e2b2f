"""ov_apply_noalloc, the entry point for callers that cannot allocate device memory,
against ov_apply: the same operator through the same kernels, with every scratch buffer
in the library's static device array instead of a workspace.

* Calls in a row on fresh contexts, the later ones on a smaller input (8^4 with two
  right-hand sides, then 4^4 with one), each equal to ov_apply bit for bit (same launch
  shape), for M, M^dag, MdagM, D_ov, D_ov^dag and H_W; the device's free memory does not
  change across the no-allocation calls (no hidden workspace).
* A call whose buffers exceed the array (16^4 multi-shift basis) and one with more
  right-hand sides than the preallocated host staging return OV_ERR_WORKSPACE.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1005_3276_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_util import CFG2, bits, dev, host, lattice, require_gpu  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def gpu():
    require_gpu(torch)


def _call(fn, lat, op, out, x, phi, nrhs):
    from paper_1005_3276_amd import _lib as L
    st = (L.OvStats * nrhs)()
    rc = getattr(L.lib(), fn)(lat._h, L.OPS[op], C.c_void_p(out.data_ptr()),
                              C.c_void_p(x.data_ptr()),
                              C.c_void_p(phi.data_ptr()) if phi is not None else None, nrhs, st)
    return rc, st


CASES = [((8, 8, 8, 8), 2, 51), ((4, 4, 4, 4), 1, 52)]  # the second input is smaller
OPS = ["m", "m_dag", "mdagm", "dov", "dov_dag", "hw"]
KW = dict(inner_tol=1e-12, **CFG2)


def test_noalloc_equals_apply_two_calls():
    from paper_1005_3276_amd import _lib as L
    # inputs, outputs and the ov_apply references first: nothing is allocated in the
    # window around the no-allocation calls except by them
    runs = []
    for dims, nrhs, seed in CASES:
        phi, src = inputs.draw(dims, nrhs=nrhs, sigma2=0.25, seed=seed)
        x, p = dev(src), dev(phi)
        ref_lat = lattice(dims, **KW)
        ref_lat.set_launch(256, 1)
        refs = {}
        for op in OPS:
            refs[op] = torch.empty_like(x)
            rc, _ = _call("ov_apply", ref_lat, op, refs[op], x, p, nrhs)
            L.check(rc, ref_lat._h)
        ref_lat.close()
        outs = {op: torch.full_like(x, float("nan")) for op in OPS}
        la = lattice(dims, **KW)
        la.set_launch(256, 1)
        runs.append((dims, nrhs, x, p, refs, outs, la))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for dims, nrhs, x, p, refs, outs, la in runs:
        for op in OPS:
            print(f"[noalloc] {dims} nrhs={nrhs} {op}", flush=True)
            rc, st = _call("ov_apply_noalloc", la, op, outs[op], x, p, nrhs)
            L.check(rc, la._h)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    print(f"[noalloc] device free memory {free0} -> {free1}", flush=True)
    assert free0 - free1 < (1 << 20), "a no-allocation call allocated device memory"
    for dims, nrhs, x, p, refs, outs, la in runs:
        for op in OPS:
            a, b = host(outs[op]), host(refs[op])
            assert np.array_equal(bits(a), bits(b)), (dims, op)
        # the binding's method is the same call
        y, _ = la.apply_noalloc("m", x, p)
        assert np.array_equal(bits(host(y)), bits(host(refs["m"]))), dims


def test_noalloc_limits():
    from paper_1005_3276_amd import _lib as L
    # 16^4: the FP64 multi-shift basis alone is ~490 MB, beyond the array
    dims = (16, 16, 16, 16)
    phi, src = inputs.draw(dims, nrhs=1, sigma2=0.25, seed=53)
    x, p = dev(src), dev(phi)
    la = lattice(dims, **KW)
    out = torch.zeros_like(x)
    rc, _ = _call("ov_apply_noalloc", la, "m", out, x, p, 1)
    msg = L.lib().ov_last_error(la._h).decode()
    print(f"[noalloc] 16^4: rc {rc} ({msg})", flush=True)
    assert rc == L.OV_ERR_WORKSPACE and "too small" in msg
    assert torch.count_nonzero(out).item() == 0  # nothing launched into out
    # more right-hand sides than the host staging set up at context creation
    dims = (4, 4, 4, 4)
    phi, src = inputs.draw(dims, nrhs=17, sigma2=0.25, seed=54)
    x, p = dev(src), dev(phi)
    la = lattice(dims, **KW)
    out = torch.zeros_like(x)
    rc, _ = _call("ov_apply_noalloc", la, "m", out, x, p, 17)
    print(f"[noalloc] nrhs 17: rc {rc} ({L.lib().ov_last_error(la._h).decode()})", flush=True)
    assert rc == L.OV_ERR_WORKSPACE
    # within both limits the same context serves the call
    y, _ = la.apply_noalloc("m", x[:2], p)
    z, _ = la.apply("m", x[:2], p)
    assert np.array_equal(bits(host(y)), bits(host(z)))
