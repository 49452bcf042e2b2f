"""Python front end: one lattice + action + solver setting on one HIP stream.

``Lattice`` wraps an ``ov_ctx``.  Fields are torch complex128 CUDA tensors of
shape ``(nrhs, T, Z, Y, X, 4)`` (or ``(T, Z, Y, X, 4)`` for one field); phi is
complex128 ``(T, Z, Y, X)``.  torch only provides device memory and the
stream; every operation is one call into libov.so.
"""
import ctypes as C

import torch

from . import _lib as L


def _stream_ptr():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Lattice:
    def __init__(self, dims, **params):
        self.params = L.default_params(dims=dims, **params)
        self.dims = tuple(dims)
        X, Y, Z, T = self.dims
        self.V = X * Y * Z * T
        self.field_shape = (T, Z, Y, X, 4)
        self.phi_shape = (T, Z, Y, X)
        h = C.c_void_p()
        L.check(L.lib().ov_ctx_create(C.byref(self.params), _stream_ptr(), C.byref(h)))
        self._h = h
        self._ws = None

    def close(self):
        if getattr(self, "_h", None):
            L.lib().ov_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ helpers
    def _check(self, status):
        L.check(status, self._h)

    def _fields(self, x):
        if x.dtype != torch.complex128 or not x.is_cuda:
            raise TypeError("fields must be complex128 CUDA tensors")
        x = x.contiguous()
        if x.shape[-5:] != self.field_shape:
            raise ValueError(f"field shape {tuple(x.shape)} does not end in {self.field_shape}")
        nrhs = 1 if x.dim() == 5 else int(torch.tensor(x.shape[:-5]).prod())
        return x, nrhs

    def _phi(self, phi):
        if phi is None:
            return None
        if phi.dtype != torch.complex128 or not phi.is_cuda or tuple(phi.shape) != self.phi_shape:
            raise TypeError(f"phi must be complex128 CUDA {self.phi_shape}")
        return phi.contiguous()

    def use_workspace(self, nrhs):
        """Allocate a caller-owned (torch) workspace for nrhs right-hand sides."""
        nbytes = L.lib().ov_workspace_bytes(self._h, nrhs)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        self._check(L.lib().ov_set_workspace(self._h, C.c_void_p(aligned), nbytes))
        return nbytes

    def coeffs(self):
        import numpy as np
        n = self.params.n_poles
        a = np.zeros(n)
        b = np.zeros(n)
        d = C.c_double()
        self._check(L.lib().ov_get_coeffs(self._h, a.ctypes.data_as(C.c_void_p),
                                          b.ctypes.data_as(C.c_void_p), C.byref(d)))
        return a, b, d.value

    def kernel_sampling(self, max_per_call):
        self._check(L.lib().ov_kernel_sampling(self._h, max_per_call))

    def kernel_times(self, kernel, reset=True):
        """(event_ms, count, bytes) of the sampled multi-shift kernel (0 t pass, 1 r pass,
        2 persistent); see kernel_spans for the device-stamped kernel-only spans."""
        return self._kernel_times(kernel, reset)[:3]

    def kernel_spans(self, kernel, reset=True):
        """(kernel_ms, count, event_ms, event_count, bytes): device-stamped spans and
        the event durations of the same sampled launches."""
        ms, cnt, by, kms, kcnt = self._kernel_times(kernel, reset)
        return kms, kcnt, ms, cnt, by

    def _kernel_times(self, kernel, reset):
        ms, by, kms = C.c_double(), C.c_double(), C.c_double()
        cnt, kcnt = C.c_longlong(), C.c_longlong()
        self._check(L.lib().ov_kernel_times(self._h, kernel, C.byref(ms), C.byref(cnt),
                                            C.byref(by), C.byref(kms), C.byref(kcnt),
                                            1 if reset else 0))
        return ms.value, cnt.value, by.value, kms.value, kcnt.value

    def set_launch(self, block=0, sites_per_thread=0):
        self._check(L.lib().ov_set_launch(self._h, block, sites_per_thread))

    def rational(self, x, phi, a0, alphas, betas):
        """a0 x + sum_i alphas_i (MdagM + betas_i)^-1 x (RHMC layers, Sec. 7.3)."""
        import numpy as np
        x, nrhs = self._fields(x)
        phi = self._phi(phi)
        al = np.ascontiguousarray(alphas, np.float64)
        be = np.ascontiguousarray(betas, np.float64)
        out = torch.empty_like(x)
        st = (L.OvStats * nrhs)()
        self._check(L.lib().ov_rational(self._h, float(a0), len(al), al.ctypes.data_as(C.c_void_p),
                                        be.ctypes.data_as(C.c_void_p), _ptr(out), _ptr(x),
                                        _ptr(phi), nrhs, st))
        return out, [s.as_dict() for s in st]

    def rational_force(self, xi, phi, a0, alphas, betas):
        """(S per rhs, G = dS/dRe phi + i dS/dIm phi summed over rhs, stats) for
        S = Re xi^dag R(MdagM) xi."""
        import numpy as np
        xi, nrhs = self._fields(xi)
        phi = self._phi(phi)
        al = np.ascontiguousarray(alphas, np.float64)
        be = np.ascontiguousarray(betas, np.float64)
        G = torch.empty(self.phi_shape, dtype=torch.complex128, device=xi.device)
        S = (C.c_double * nrhs)()
        st = (L.OvStats * nrhs)()
        self._check(L.lib().ov_rational_force(self._h, float(a0), len(al),
                                              al.ctypes.data_as(C.c_void_p),
                                              be.ctypes.data_as(C.c_void_p), _ptr(G), S,
                                              _ptr(xi), _ptr(phi), nrhs, st))
        return list(S), G, [s.as_dict() for s in st]

    def boson(self, phi):
        """(S_B, G_B, F) of the bosonic action of eq. acws (see ov_boson)."""
        phi = self._phi(phi)
        G = torch.empty(self.phi_shape, dtype=torch.complex128, device=phi.device)
        F = torch.empty_like(G)
        S = C.c_double()
        self._check(L.lib().ov_boson(self._h, _ptr(phi), C.byref(S), _ptr(G), _ptr(F)))
        return S.value, G, F

    def rhmc_trajectory(self, phi, pi, R, nsteps, tau, c18, c14, u):
        """One RHMC trajectory; phi is updated in place when accepted.
        c18, c14: (a0, alphas, betas) of x^{1/8} and x^{-1/4}.  Returns (dH, accepted)."""
        import numpy as np
        phi = self._phi(phi)
        pi = self._phi(pi)
        R, nrhs = self._fields(R)
        if nrhs != 1:
            raise ValueError("one pseudofermion field")
        a18, al18, be18 = float(c18[0]), np.ascontiguousarray(c18[1], np.float64), np.ascontiguousarray(c18[2], np.float64)
        a14, al14, be14 = float(c14[0]), np.ascontiguousarray(c14[1], np.float64), np.ascontiguousarray(c14[2], np.float64)
        dH = C.c_double()
        acc = C.c_int()
        st = L.OvStats()
        vp = lambda a: a.ctypes.data_as(C.c_void_p)
        self._check(L.lib().ov_rhmc_trajectory(self._h, _ptr(phi), _ptr(pi), _ptr(R), nsteps,
                                               float(tau), a18, len(al18), vp(al18), vp(be18),
                                               a14, len(al14), vp(al14), vp(be14), float(u),
                                               C.byref(dH), C.byref(acc), C.byref(st)))
        return dH.value, bool(acc.value)

    def locality(self, spin=0):
        """Locality probe of Sec. 3.2 for this lattice's Dirac form: f(r) for
        r = 0 .. sum L/2 (numpy array) and the stats dict."""
        import numpy as np
        nr = sum(d // 2 for d in self.dims) + 1
        f = np.zeros(nr)
        st = L.OvStats()
        self._check(L.lib().ov_locality(self._h, spin, f.ctypes.data_as(C.c_void_p), nr,
                                        C.byref(st)))
        return f, st.as_dict()

    # --------------------------------------------------------- operations
    def sign(self, x):
        x, nrhs = self._fields(x)
        out = torch.empty_like(x)
        st = (L.OvStats * nrhs)()
        self._check(L.lib().ov_sign(self._h, _ptr(out), _ptr(x), nrhs, st))
        return out, [s.as_dict() for s in st]

    def apply(self, op, x, phi=None):
        x, nrhs = self._fields(x)
        phi = self._phi(phi)
        out = torch.empty_like(x)
        st = (L.OvStats * nrhs)()
        code = L.OPS[op] if isinstance(op, str) else int(op)
        self._check(L.lib().ov_apply(self._h, code, _ptr(out), _ptr(x),
                                     _ptr(phi) if phi is not None else None, nrhs, st))
        return out, [s.as_dict() for s in st]

    def apply_noalloc(self, op, x, phi=None):
        """apply() through ov_apply_noalloc: the library allocates nothing (its scratch
        is a static device array of OV_NOALLOC_SCRATCH_BYTES; see include/ov.h)."""
        x, nrhs = self._fields(x)
        phi = self._phi(phi)
        out = torch.empty_like(x)
        st = (L.OvStats * nrhs)()
        code = L.OPS[op] if isinstance(op, str) else int(op)
        self._check(L.lib().ov_apply_noalloc(self._h, code, _ptr(out), _ptr(x),
                                             _ptr(phi) if phi is not None else None, nrhs, st))
        return out, [s.as_dict() for s in st]

    def solve(self, b, phi, x0=None):
        b, nrhs = self._fields(b)
        phi = self._phi(phi)
        x = torch.zeros_like(b) if x0 is None else x0.clone().contiguous()
        st = (L.OvStats * nrhs)()
        status = L.lib().ov_solve(self._h, _ptr(x), _ptr(b), _ptr(phi), nrhs, st)
        stats = [s.as_dict() for s in st]
        if status == L.OV_ERR_NOT_CONVERGED:
            raise L.OvError(status, f"not converged: {stats}")
        self._check(status)
        return x, stats

    def force(self, xi, phi):
        xi, nrhs = self._fields(xi)
        phi = self._phi(phi)
        G = torch.empty(self.phi_shape, dtype=torch.complex128, device=xi.device)
        S = (C.c_double * nrhs)()
        st = (L.OvStats * nrhs)()
        self._check(L.lib().ov_force(self._h, _ptr(G), S, _ptr(xi), _ptr(phi), nrhs, st))
        return [S[i] for i in range(nrhs)], G, [s.as_dict() for s in st]

    def stencil_bench(self, x_planar, prec, reps=10):
        """out = H_W x on a spin-planar field (complex64/complex128 (nrhs, 4, V))."""
        nrhs = x_planar.shape[0]
        out = torch.empty_like(x_planar)
        ms = C.c_float()
        self._check(L.lib().ov_stencil_bench(self._h, prec, _ptr(out), _ptr(x_planar), nrhs,
                                             reps, C.byref(ms)))
        return out, ms.value

    def pack(self, x, prec):
        x, nrhs = self._fields(x)
        dt = torch.complex64 if prec else torch.complex128
        out = torch.empty((nrhs, 4, self.V), dtype=dt, device=x.device)
        self._check(L.lib().ov_pack(self._h, prec, _ptr(out), _ptr(x), nrhs))
        return out

    def unpack(self, xp, prec):
        nrhs = xp.shape[0]
        out = torch.empty((nrhs,) + self.field_shape, dtype=torch.complex128, device=xp.device)
        xp = xp.contiguous()  # held until the call has been enqueued
        self._check(L.lib().ov_unpack(self._h, prec, _ptr(out), _ptr(xp), nrhs))
        return out


def solve_batch(lattices, bs, phis):
    """Solve every (lattice, b, phi) in one batched launch sequence."""
    n = len(lattices)
    ctx = (C.c_void_p * n)(*[l._h.value for l in lattices])
    bl, xl, pl, nr = [], [], [], []
    xs, held = [], []  # every tensor whose pointer is passed stays referenced until the call
    for lat, b, phi in zip(lattices, bs, phis):
        b, nrhs = lat._fields(b)
        phi = lat._phi(phi)
        x = torch.zeros_like(b)
        xs.append(x)
        held += [b, phi]
        bl.append(b.data_ptr())
        xl.append(x.data_ptr())
        pl.append(phi.data_ptr())
        nr.append(nrhs)
    tot = sum(nr)
    st = (L.OvStats * tot)()
    status = L.lib().ov_solve_batch(n, ctx, (C.c_void_p * n)(*xl), (C.c_void_p * n)(*bl),
                                    (C.c_void_p * n)(*pl), (C.c_int * n)(*nr), st)
    if status == L.OV_ERR_NOT_CONVERGED:
        raise L.OvError(status, f"not converged: {[s.as_dict() for s in st]}")
    L.check(status, lattices[0]._h)
    return xs, [s.as_dict() for s in st]
