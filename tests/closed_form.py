"""Momentum-space closed forms of the free Wilson / overlap operators (pins).

The theory has no gauge field, so every operator on the path is diagonal in
momentum space (Sec. 7.2 applies the Dirac operator that way).  These helpers
build it from the paper's own momentum-space functions, independently of the
position-space stencil:

  * M(p) = 1 - 2 sum_mu sin^2(p_mu/2),  s(p) = sqrt(sum_mu sin^2 p_mu + M(p)^2)
    (Sec. 4.1, one-loop definitions);
  * D_W(-1)(p) = -M(p) + i sum_mu gamma_mu sin p_mu for fields ~ exp(+i p.x),
    i.e. A(p) = M + ... with the paper's (1 - a D_2/2)(p) = 1/2 + M/(2s) and
    D_1(p) ~ gamma.sin p / s (Sec. 3.1, mode analysis);
  * antiperiodic time: p_t = (2n+1) pi / T (Sec. 3.1).

gamma matrices are the paper's (Sec. 2.1), written here from their definition.
"""
import numpy as np

S1 = np.array([[0, 1], [1, 0]], complex)
S2 = np.array([[0, -1j], [1j, 0]], complex)
S3 = np.array([[1, 0], [0, -1]], complex)
Z2 = np.zeros((2, 2), complex)
I2 = np.eye(2, dtype=complex)


def paper_gammas():
    """(g_x, g_y, g_z, g_t, g5) in the paper's basis."""
    gi = [np.block([[Z2, 1j * s], [-1j * s, Z2]]) for s in (S1, S2, S3)]
    g0 = np.block([[Z2, I2], [I2, Z2]])
    g5 = np.block([[-I2, Z2], [Z2, I2]])
    return gi[0], gi[1], gi[2], g0, g5


def momenta(dims, bc_t=-1):
    """Momentum grids p_mu for numpy's FFT ordering, arrays shaped (T,Z,Y,X)."""
    X, Y, Z, T = dims
    px = 2 * np.pi * np.fft.fftfreq(X) * 1.0
    py = 2 * np.pi * np.fft.fftfreq(Y)
    pz = 2 * np.pi * np.fft.fftfreq(Z)
    pt = 2 * np.pi * np.fft.fftfreq(T)
    if bc_t == -1:
        pt = pt + np.pi / T
    PT, PZ, PY, PX = np.meshgrid(pt, pz, py, px, indexing="ij")
    return PX, PY, PZ, PT


def M_s(dims, bc_t=-1):
    PX, PY, PZ, PT = momenta(dims, bc_t)
    ps = (PX, PY, PZ, PT)
    Mp = 1 - 2 * sum(np.sin(p / 2) ** 2 for p in ps)
    sin2 = sum(np.sin(p) ** 2 for p in ps)
    s = np.sqrt(sin2 + Mp ** 2)
    return Mp, np.sqrt(sin2), s


def hw_symbol(dims, bc_t=-1, M0=1.0):
    """H_W(p) = g5 [ (4 - M0 - sum cos p) + i sum gamma_mu sin p_mu ], shape (T,Z,Y,X,4,4)."""
    gx, gy, gz, gt, g5 = paper_gammas()
    PX, PY, PZ, PT = momenta(dims, bc_t)
    diag = 4 - M0 - (np.cos(PX) + np.cos(PY) + np.cos(PZ) + np.cos(PT))
    D = diag[..., None, None] * np.eye(4)
    for p, g in ((PX, gx), (PY, gy), (PZ, gz), (PT, gt)):
        D = D + 1j * np.sin(p)[..., None, None] * g
    return np.einsum("ab,...bc->...ac", g5, D)


def _to_mom(field, dims, bc_t):
    X, Y, Z, T = dims
    f = np.asarray(field).reshape(T, Z, Y, X, 4)
    if bc_t == -1:
        t = np.arange(T)
        f = f * np.exp(-1j * np.pi * t / T)[:, None, None, None, None]
    return np.fft.fftn(f, axes=(0, 1, 2, 3))


def _from_mom(fh, dims, bc_t):
    X, Y, Z, T = dims
    f = np.fft.ifftn(fh, axes=(0, 1, 2, 3))
    if bc_t == -1:
        t = np.arange(T)
        f = f * np.exp(1j * np.pi * t / T)[:, None, None, None, None]
    return f


def apply_symbol(symbol, field, dims, bc_t=-1):
    """Apply a momentum-space 4x4 symbol (T,Z,Y,X,4,4) to a position-space field."""
    fh = _to_mom(field, dims, bc_t)
    gh = np.einsum("...ab,...b->...a", symbol, fh)
    return _from_mom(gh, dims, bc_t)


def rational_symbol(dims, a, b, bc_t=-1):
    """r(H_W)(p) = H_W(p) sum_k a_k / (s^2 + b_k)   (H_W(p)^2 = s(p)^2)."""
    H = hw_symbol(dims, bc_t)
    _, _, s = M_s(dims, bc_t)
    R = sum(ak / (s ** 2 + bk) for ak, bk in zip(a, b))
    return H * R[..., None, None]


def exact_sign_symbol(dims, bc_t=-1):
    H = hw_symbol(dims, bc_t)
    _, _, s = M_s(dims, bc_t)
    return H / s[..., None, None]


def dov_symbol(sign_sym):
    g5 = paper_gammas()[4]
    return np.eye(4) + np.einsum("ab,...bc->...ac", g5, sign_sym)


def dense_from_symbol(symbol, dims, bc_t=-1):
    """Dense (4V x 4V) position-space matrix of a momentum-space symbol."""
    X, Y, Z, T = dims
    n = 4 * X * Y * Z * T
    out = np.empty((n, n), complex)
    e = np.zeros(n, complex)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        out[:, j] = apply_symbol(symbol, e, dims, bc_t).reshape(-1)
    return out


def yukawa_dense(phi, m, g, dag=False):
    """Dense site-local c+ P+ + c- P- (or its adjoint), natural layout."""
    g5 = paper_gammas()[4]
    Pp = 0.5 * (np.eye(4) + g5)
    Pm = 0.5 * (np.eye(4) - g5)
    phi = np.asarray(phi).reshape(-1)
    V = phi.size
    Yd = np.zeros((4 * V, 4 * V), complex)
    for x in range(V):
        cp = m + g * phi[x]
        cm = np.conj(m) + np.conj(g) * np.conj(phi[x])
        blk = cp * Pp + cm * Pm
        if dag:
            blk = blk.conj().T
        Yd[4 * x: 4 * x + 4, 4 * x: 4 * x + 4] = blk
    return Yd
