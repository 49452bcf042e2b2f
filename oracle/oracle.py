"""ctypes wrapper of the plain FP64 C oracle (TEST INFRASTRUCTURE ONLY).

Every function takes and returns numpy arrays in the natural layout:
fields are complex128 ``(T, Z, Y, X, 4)`` (or flat ``V*4``), phi is complex128
``(T, Z, Y, X)``.  The arithmetic lives in ``ov_oracle.c``; this module only
marshals arguments.  Operator conventions are stated in ``ov_oracle.h``.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(HERE, "libovoracle.so")
MAX_POLES = 64

OP_HW, OP_DOV, OP_DOV_DAG, OP_M, OP_M_DAG, OP_MDAGM = range(6)
# forms of the Dirac operator inside M (ov_oracle.h, ORC_DIRAC_*)
DIRAC_OVERLAP_MS, DIRAC_OVERLAP_RAT, DIRAC_OVERLAP_EXACT, DIRAC_DSLASH = range(4)


class Params(C.Structure):
    _fields_ = [("dims", C.c_int * 4), ("bc_t", C.c_int), ("M0", C.c_double),
                ("m_re", C.c_double), ("m_im", C.c_double),
                ("g_re", C.c_double), ("g_im", C.c_double),
                ("n_poles", C.c_int), ("lambda_min", C.c_double),
                ("lambda_max", C.c_double), ("inner_tol", C.c_double),
                ("max_inner", C.c_int),
                ("a", C.c_double * MAX_POLES), ("b", C.c_double * MAX_POLES),
                ("delta", C.c_double), ("d0", C.c_double), ("dirac", C.c_int)]


class MsStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("max_shift_res", C.c_double)]


class CgStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int),
                ("inner_iters", C.c_longlong), ("true_rel_res", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            from . import build as _b
            _b.build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        L.orc_gamma.argtypes = [C.c_int, P]
        L.orc_zolotarev.argtypes = [C.c_int, C.c_double, C.c_double, P, P, P, P]
        L.orc_sncndn.argtypes = [C.c_double, C.c_double, P, P, P, P]
        L.orc_sncndn.restype = None
        L.orc_init.argtypes = [P]
        L.orc_dw.argtypes = [P, P, P]
        L.orc_dw.restype = None
        L.orc_hw.argtypes = [P, P, P]
        L.orc_hw.restype = None
        L.orc_multishift.argtypes = [P, C.c_int, P, P, C.c_double, C.c_int, P, P, P, P]
        L.orc_sign.argtypes = [P, P, P, P]
        L.orc_apply.argtypes = [P, C.c_int, P, P, P, P]
        L.orc_solve.argtypes = [P, P, P, P, C.c_double, C.c_int, P]
        L.orc_force.argtypes = [P, P, P, C.c_double, C.c_int, P, P, P]
        L.orc_residual.argtypes = [P, P, P, P]
        L.orc_residual.restype = C.c_double
        L.orc_threads.restype = C.c_int
        L.orc_m0inv.argtypes = [P, C.c_int, P, P, C.c_double, C.c_int]
        L.orc_locality.argtypes = [P, C.c_int, P, C.c_int]
        L.orc_rational.argtypes = [P, P, C.c_double, C.c_int, P, P, P, P, C.c_double, C.c_int]
        L.orc_boson.argtypes = [P, P, P, P, P]
        L.orc_rhmc_trajectory.argtypes = [P, P, P, P, C.c_int, C.c_double, C.c_double, C.c_int,
                                          P, P, C.c_double, C.c_int, P, P, C.c_double,
                                          C.c_double, C.c_int, P, P]
        L.orc_rhmc_trajectory_ex.argtypes = [P, P, P, P, C.c_int, C.c_double, C.c_double,
                                             C.c_int, P, P, C.c_double, C.c_int, P, P,
                                             C.c_double, C.c_double, C.c_int, P, P, P, P]
        L.orc_rational_force.argtypes = [P, P, C.c_double, C.c_int, P, P, P, C.c_double,
                                         C.c_int, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


class Oracle:
    """One lattice + action + sign-approximation setting."""

    def __init__(self, dims, bc_t=-1, M0=1.0, m=0.05, g=0.1, n_poles=16,
                 lambda_min=0.01, lambda_max=8.0, inner_tol=1e-13, max_inner=5000,
                 dirac=DIRAC_OVERLAP_MS):
        p = Params()
        X, Y, Z, T = dims
        p.dims[:] = [X, Y, Z, T]
        p.bc_t = bc_t
        p.M0 = M0
        m = complex(m)
        g = complex(g)
        p.m_re, p.m_im, p.g_re, p.g_im = m.real, m.imag, g.real, g.imag
        p.n_poles = n_poles
        p.lambda_min, p.lambda_max = lambda_min, lambda_max
        p.inner_tol, p.max_inner = inner_tol, max_inner
        p.dirac = dirac
        rc = lib().orc_init(C.byref(p))
        if rc != 0:
            raise ValueError(f"orc_init failed ({rc})")
        self.p = p
        self.dims = (X, Y, Z, T)
        self.V = X * Y * Z * T
        self.shape = (T, Z, Y, X, 4)

    # --- coefficients
    @property
    def a(self):
        return np.array(self.p.a[: self.p.n_poles])

    @property
    def b(self):
        return np.array(self.p.b[: self.p.n_poles])

    @property
    def delta(self):
        return self.p.delta

    def set_inner_tol(self, tol):
        self.p.inner_tol = tol

    # --- operators
    def _field(self, v):
        v = _c128(v)
        assert v.size == 4 * self.V, (v.shape, self.shape)
        return v

    def _phi(self, phi):
        if phi is None:
            return np.zeros(self.V, np.complex128)
        phi = _c128(phi)
        assert phi.size == self.V
        return phi

    def dw(self, v):
        v = self._field(v)
        out = np.empty_like(v)
        lib().orc_dw(C.byref(self.p), _ptr(v), _ptr(out))
        return out.reshape(v.shape)

    def hw(self, v):
        v = self._field(v)
        out = np.empty_like(v)
        lib().orc_hw(C.byref(self.p), _ptr(v), _ptr(out))
        return out.reshape(v.shape)

    def multishift(self, src, shifts, coef=None, tol=None, maxit=None, want_ys=False):
        src = self._field(src)
        shifts = np.ascontiguousarray(shifts, np.float64)
        n = len(shifts)
        acc = np.zeros_like(src) if coef is not None else None
        cf = np.ascontiguousarray(coef, np.float64) if coef is not None else None
        ys = np.zeros((n,) + src.shape, np.complex128) if want_ys else None
        st = MsStats()
        rc = lib().orc_multishift(C.byref(self.p), n, _ptr(shifts),
                                  _ptr(cf) if cf is not None else None,
                                  tol if tol is not None else self.p.inner_tol,
                                  maxit if maxit is not None else self.p.max_inner,
                                  _ptr(src), _ptr(acc) if acc is not None else None,
                                  _ptr(ys) if ys is not None else None, C.byref(st))
        return acc, ys, st, rc

    def sign(self, v):
        v = self._field(v)
        out = np.empty_like(v)
        st = MsStats()
        rc = lib().orc_sign(C.byref(self.p), _ptr(v), _ptr(out), C.byref(st))
        if rc != 0:
            raise RuntimeError(f"orc_sign did not converge ({rc})")
        return out.reshape(v.shape), st

    def apply(self, op, v, phi=None):
        v = self._field(v)
        ph = self._phi(phi)
        out = np.empty_like(v)
        inner = C.c_longlong(0)
        rc = lib().orc_apply(C.byref(self.p), op, _ptr(ph), _ptr(v), _ptr(out), C.byref(inner))
        if rc != 0:
            raise RuntimeError(f"orc_apply({op}) failed ({rc})")
        return out.reshape(v.shape)

    def solve(self, b, phi, tol=1e-10, maxit=2000):
        b = self._field(b)
        ph = self._phi(phi)
        x = np.empty_like(b)
        st = CgStats()
        rc = lib().orc_solve(C.byref(self.p), _ptr(ph), _ptr(b), _ptr(x), tol, maxit,
                             C.byref(st))
        return x.reshape(b.shape), st, rc

    def force(self, phi, xi, tol=1e-12, maxit=2000):
        xi = self._field(xi)
        ph = self._phi(phi)
        G = np.empty(self.V, np.complex128)
        S = C.c_double(0.0)
        st = CgStats()
        rc = lib().orc_force(C.byref(self.p), _ptr(ph), _ptr(xi), tol, maxit, C.byref(S),
                             _ptr(G), C.byref(st))
        return S.value, G.reshape(self.shape[:4]), st, rc

    def m0inv(self, v, dag=False, tol=1e-13, maxit=4000):
        """M0^-1 v (or M0^-dag v), M0 = M at phi = 0: the free-field
        preconditioner of Sec. 7.3, from its definition by CG."""
        v = self._field(v)
        out = np.empty_like(v)
        rc = lib().orc_m0inv(C.byref(self.p), 1 if dag else 0, _ptr(v), _ptr(out), tol, maxit)
        if rc != 0:
            raise RuntimeError(f"orc_m0inv did not converge ({rc})")
        return out.reshape(v.shape)

    def rational(self, v, phi, a0, alpha, beta, tol=1e-12, maxit=4000):
        """a0 v + sum_i alpha_i (MdagM + beta_i)^-1 v, one CG per shift (Sec. 7.3)."""
        v = self._field(v)
        ph = self._phi(phi)
        al = np.ascontiguousarray(alpha, np.float64)
        be = np.ascontiguousarray(beta, np.float64)
        out = np.empty_like(v)
        rc = lib().orc_rational(C.byref(self.p), _ptr(ph), a0, len(al), _ptr(al), _ptr(be),
                                _ptr(v), _ptr(out), tol, maxit)
        if rc != 0:
            raise RuntimeError(f"orc_rational did not converge ({rc})")
        return out.reshape(v.shape)

    def rational_force(self, phi, xi, a0, alpha, beta, tol=1e-12, maxit=4000):
        xi = self._field(xi)
        ph = self._phi(phi)
        al = np.ascontiguousarray(alpha, np.float64)
        be = np.ascontiguousarray(beta, np.float64)
        G = np.empty(self.V, np.complex128)
        S = C.c_double(0.0)
        rc = lib().orc_rational_force(C.byref(self.p), _ptr(ph), a0, len(al), _ptr(al),
                                      _ptr(be), _ptr(xi), tol, maxit, C.byref(S), _ptr(G))
        if rc != 0:
            raise RuntimeError(f"orc_rational_force did not converge ({rc})")
        return S.value, G.reshape(self.shape[:4])

    def boson(self, phi):
        """(S_B, G_B, F) of the bosonic action of eq. acws (Sec. 7.3)."""
        ph = np.ascontiguousarray(phi, np.complex128).reshape(-1)
        G = np.empty(self.V, np.complex128)
        F = np.empty(self.V, np.complex128)
        S = C.c_double(0.0)
        lib().orc_boson(C.byref(self.p), _ptr(ph), C.byref(S), _ptr(G), _ptr(F))
        return S.value, G.reshape(self.shape[:4]), F.reshape(self.shape[:4])

    def rhmc_trajectory(self, phi, pi, R, nsteps, tau, c18, c14, u, tol=1e-12, maxit=4000,
                        start=False):
        """One RHMC trajectory; returns (phi_end_or_start, dH, accepted), and with
        start=True also (eta, H_parts): the heatbath field eta = r18(MdagM) R and the
        kinetic, bosonic and pseudofermion parts of H at the start."""
        ph = np.ascontiguousarray(phi, np.complex128).reshape(-1).copy()
        pi = np.ascontiguousarray(pi, np.complex128).reshape(-1)
        R = self._field(R)
        a18, al18, be18 = c18[0], np.ascontiguousarray(c18[1], np.float64), np.ascontiguousarray(c18[2], np.float64)
        a14, al14, be14 = c14[0], np.ascontiguousarray(c14[1], np.float64), np.ascontiguousarray(c14[2], np.float64)
        dH = C.c_double(0.0)
        acc = C.c_int(0)
        eta = np.zeros_like(R)
        parts = np.zeros(3)
        rc = lib().orc_rhmc_trajectory_ex(C.byref(self.p), _ptr(ph), _ptr(pi), _ptr(R), nsteps,
                                          tau, a18, len(al18), _ptr(al18), _ptr(be18), a14,
                                          len(al14), _ptr(al14), _ptr(be14), u, tol, maxit,
                                          C.byref(dH), C.byref(acc), _ptr(eta), _ptr(parts))
        if rc != 0:
            raise RuntimeError(f"orc_rhmc_trajectory: a solve did not converge ({rc})")
        out = (ph.reshape(self.shape[:4]), dH.value, bool(acc.value))
        if start:
            return out + (eta.reshape(self.shape), parts)
        return out

    def locality(self, spin=0):
        """f(r), r = 0 .. sum L/2, of the locality probe of Sec. 3.2 for this D."""
        nr = sum(d // 2 for d in self.dims) + 1
        f = np.zeros(nr)
        rc = lib().orc_locality(C.byref(self.p), spin, _ptr(f), nr)
        if rc != 0:
            raise RuntimeError(f"orc_locality failed ({rc})")
        return f

    def residual(self, b, x, phi):
        b = self._field(b)
        x = self._field(x)
        ph = self._phi(phi)
        return lib().orc_residual(C.byref(self.p), _ptr(ph), _ptr(b), _ptr(x))


def gamma(mu):
    out = np.zeros(16, np.complex128)
    lib().orc_gamma(mu, _ptr(out))
    return out.reshape(4, 4)


def zolotarev(n, lmin, lmax):
    a = np.zeros(n)
    b = np.zeros(n)
    delta = C.c_double()
    d0 = C.c_double()
    rc = lib().orc_zolotarev(n, lmin, lmax, _ptr(a), _ptr(b), C.byref(delta), C.byref(d0))
    if rc != 0:
        raise ValueError("orc_zolotarev failed")
    return a, b, delta.value, d0.value


def sncndn(u, m1):
    vals = [C.c_double() for _ in range(4)]
    lib().orc_sncndn(u, m1, *[C.byref(v) for v in vals])
    return tuple(v.value for v in vals)


def threads():
    return lib().orc_threads()
