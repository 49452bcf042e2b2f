"""ctypes binding of libov.so (argument marshalling only).

Every step of the computation runs in the HIP library; this module converts
torch tensors to device pointers and the current HIP stream, and raises on
any non-OK status.  It fails loudly when the library has not been built.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libov.so")

OV_OK, OV_ERR_INVALID_ARG, OV_ERR_NOT_CONVERGED, OV_ERR_BREAKDOWN, OV_ERR_SPECTRUM, \
    OV_ERR_WORKSPACE, OV_ERR_DEVICE = range(7)
OV_FP64, OV_MIXED = 0, 1
OP_HW, OP_DOV, OP_DOV_DAG, OP_M, OP_M_DAG, OP_MDAGM, OP_M0INV, OP_M0INV_DAG = range(8)
DIRAC_OVERLAP_MS, DIRAC_OVERLAP_RAT, DIRAC_OVERLAP_EXACT, DIRAC_DSLASH = range(4)
DIRACS = {"overlap": DIRAC_OVERLAP_MS, "overlap_rat": DIRAC_OVERLAP_RAT,
          "overlap_exact": DIRAC_OVERLAP_EXACT, "dslash": DIRAC_DSLASH}
OPS = {"hw": OP_HW, "dov": OP_DOV, "dov_dag": OP_DOV_DAG, "m": OP_M, "m_dag": OP_M_DAG,
       "mdagm": OP_MDAGM, "m0inv": OP_M0INV, "m0inv_dag": OP_M0INV_DAG}

# every symbol include/ov.h declares
SYMBOLS = ["ov_params_default", "ov_ctx_create", "ov_ctx_destroy", "ov_workspace_bytes",
           "ov_workspace_bytes_rational",
           "ov_set_workspace", "ov_get_coeffs", "ov_zolotarev", "ov_sign", "ov_apply",
           "ov_apply_noalloc", "ov_solve", "ov_solve_batch", "ov_force", "ov_stencil_bench", "ov_pack",
           "ov_unpack", "ov_set_launch", "ov_get_launch", "ov_tune_ms", "ov_kernel_sampling",
           "ov_kernel_times", "ov_locality", "ov_rational", "ov_rational_force", "ov_boson",
           "ov_rhmc_trajectory",
           "ov_status_string", "ov_last_error"]


class OvParams(C.Structure):
    _fields_ = [("dims", C.c_int * 4), ("bc_t", C.c_int), ("M0", C.c_double),
                ("m_re", C.c_double), ("m_im", C.c_double),
                ("g_re", C.c_double), ("g_im", C.c_double),
                ("n_poles", C.c_int), ("lambda_min", C.c_double), ("lambda_max", C.c_double),
                ("inner_tol", C.c_double), ("outer_tol", C.c_double),
                ("truth_tol", C.c_double), ("mixed_inner_tol", C.c_double),
                ("reliable_delta", C.c_double), ("max_inner", C.c_int),
                ("max_outer", C.c_int), ("precision", C.c_int),
                ("inner_relax", C.c_double), ("inner_tol_max", C.c_double),
                ("precondition", C.c_int), ("dirac", C.c_int), ("truth_relax", C.c_double),
                ("inner_form", C.c_int), ("pc_mass", C.c_int), ("shift_pc_cutoff", C.c_double)]


class OvStats(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("reliable_updates", C.c_int),
                ("inner_iters", C.c_longlong), ("stencil_apps", C.c_longlong),
                ("true_rel_res", C.c_double), ("max_shift_res", C.c_double),
                ("seconds", C.c_double), ("model_bytes", C.c_double),
                ("stagnations", C.c_int), ("fp64_fallback", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class OvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load libov.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            raise ImportError(f"{SO} not built: run __graft_entry__.build() or "
                              "python paper_1005_3276_amd/build.py")
        L = C.CDLL(SO)
        P = C.c_void_p
        L.ov_params_default.argtypes = [P]
        L.ov_params_default.restype = None
        L.ov_ctx_create.argtypes = [P, P, C.POINTER(P)]
        L.ov_ctx_destroy.argtypes = [P]
        L.ov_workspace_bytes.argtypes = [P, C.c_int]
        L.ov_workspace_bytes.restype = C.c_size_t
        L.ov_workspace_bytes_rational.argtypes = [P, C.c_int, C.c_int]
        L.ov_workspace_bytes_rational.restype = C.c_size_t
        L.ov_set_workspace.argtypes = [P, P, C.c_size_t]
        L.ov_get_coeffs.argtypes = [P, P, P, P]
        L.ov_zolotarev.argtypes = [C.c_int, C.c_double, C.c_double, P, P, P]
        L.ov_sign.argtypes = [P, P, P, C.c_int, P]
        L.ov_apply.argtypes = [P, C.c_int, P, P, P, C.c_int, P]
        L.ov_apply_noalloc.argtypes = [P, C.c_int, P, P, P, C.c_int, P]
        L.ov_solve.argtypes = [P, P, P, P, C.c_int, P]
        L.ov_solve_batch.argtypes = [C.c_int, P, P, P, P, P, P]
        L.ov_force.argtypes = [P, P, P, P, P, C.c_int, P]
        L.ov_stencil_bench.argtypes = [P, C.c_int, P, P, C.c_int, C.c_int, P]
        L.ov_pack.argtypes = [P, C.c_int, P, P, C.c_int]
        L.ov_unpack.argtypes = [P, C.c_int, P, P, C.c_int]
        L.ov_set_launch.argtypes = [P, C.c_int, C.c_int]
        L.ov_get_launch.argtypes = [P, P, P]
        L.ov_tune_ms.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P]
        L.ov_kernel_sampling.argtypes = [P, C.c_int]
        L.ov_kernel_times.argtypes = [P, C.c_int, P, P, P, P, P, C.c_int]
        L.ov_locality.argtypes = [P, C.c_int, P, C.c_int, P]
        L.ov_rational.argtypes = [P, C.c_double, C.c_int, P, P, P, P, P, C.c_int, P]
        L.ov_rational_force.argtypes = [P, C.c_double, C.c_int, P, P, P, P, P, P, C.c_int, P]
        L.ov_boson.argtypes = [P, P, P, P, P]
        L.ov_rhmc_trajectory.argtypes = [P, P, P, P, C.c_int, C.c_double, C.c_double, C.c_int,
                                         P, P, C.c_double, C.c_int, P, P, C.c_double, P, P, P]
        L.ov_status_string.argtypes = [C.c_int]
        L.ov_status_string.restype = C.c_char_p
        L.ov_last_error.argtypes = [P]
        L.ov_last_error.restype = C.c_char_p
        for fn in ("ov_ctx_create", "ov_ctx_destroy", "ov_set_workspace", "ov_get_coeffs",
                   "ov_zolotarev", "ov_sign", "ov_apply", "ov_apply_noalloc", "ov_solve",
                   "ov_solve_batch",
                   "ov_force", "ov_stencil_bench", "ov_pack", "ov_unpack", "ov_set_launch",
                   "ov_get_launch", "ov_tune_ms", "ov_kernel_sampling", "ov_kernel_times",
                   "ov_locality", "ov_rational", "ov_rational_force", "ov_boson",
                   "ov_rhmc_trajectory"):
            getattr(L, fn).restype = C.c_int
        _lib = L
    return _lib


def check(status, ctx=None):
    if status != OV_OK:
        L = lib()
        msg = L.ov_last_error(ctx).decode() if ctx is not None else L.ov_last_error(None).decode()
        raise OvError(status, f"{L.ov_status_string(status).decode()}: {msg}")


_PARAM_FIELDS = {f[0] for f in OvParams._fields_}


def default_params(**kw) -> OvParams:
    p = OvParams()
    lib().ov_params_default(C.byref(p))
    for k, v in kw.items():
        if k == "dims":
            p.dims[:] = list(v)
        elif k in ("m", "g"):
            v = complex(v)
            setattr(p, k + "_re", v.real)
            setattr(p, k + "_im", v.imag)
        elif k == "precision":
            p.precision = {"fp64": OV_FP64, "mixed": OV_MIXED}.get(v, v)
        elif k == "dirac":
            p.dirac = DIRACS.get(v, v)
        elif k in _PARAM_FIELDS:
            setattr(p, k, v)
        else:
            raise TypeError(f"unknown ov_params field {k!r}")
    return p


def zolotarev(n, lmin, lmax):
    import numpy as np
    a = np.zeros(n)
    b = np.zeros(n)
    d = C.c_double()
    check(lib().ov_zolotarev(n, lmin, lmax, a.ctypes.data_as(C.c_void_p),
                             b.ctypes.data_as(C.c_void_p), C.byref(d)))
    return a, b, d.value
