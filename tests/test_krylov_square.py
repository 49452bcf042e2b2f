"""Method check (CPU, numpy) of the second function the GPU takes from one multi-shift.

The FP64 true residual of the solver needs eps^2 x = A r(A)^2 x (A = H^2, r the
Zolotarev pole sum) and takes it from the Krylov space that the multi-shift CG for
eps(x) = H r(A) x builds: with the CG scalars alpha_j, rho_j the Lanczos tridiagonal of
A is T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_j,j+1 = sqrt(beta_j)/alpha_j on
v_j = (-1)^j r_j / |r_j|, and r(A)^2 x ~ |x| V r(T)^2 e_1.  This test runs that recipe
in plain numpy (dense random Hermitian H with the free-field spectral range |H| in
[1, 7], the 20-pole coefficients of the solver) and checks it against the dense
eigendecomposition, together with the accuracy the solver assumes (about ten times the
multi-shift tolerance).
"""
import numpy as np
import pytest


def _krylov(H, x, tol):
    """CG on A = H^2 from r_0 = x until |r_N| <= tol |x| (the stop of its smallest shift,
    whose zeta factor is ~1): scalars alpha_j, rho_j and the residuals r_j."""
    r = x.copy()
    rho = [np.vdot(r, r).real]
    alpha, rs, p = [], [], None
    while np.sqrt(rho[-1] / rho[0]) > tol and len(alpha) < 400:
        rs.append(r.copy())
        p = r.copy() if p is None else r + (rho[-1] / rho[-2]) * p
        q = H @ (H @ p)
        alpha.append(rho[-1] / np.vdot(p, q).real)
        r = r - alpha[-1] * q
        rho.append(np.vdot(r, r).real)
    return np.array(alpha), np.array(rho), rs


@pytest.mark.parametrize("tol", [1e-8, 1e-12])
def test_eps_squared_from_krylov_space(tol):
    from paper_1005_3276_amd import _lib
    rng = np.random.default_rng(7)
    n = 300
    ev = np.concatenate([rng.uniform(1, 7, n // 2), -rng.uniform(1, 7, n - n // 2)])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    H = (Q * ev) @ Q.conj().T
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a, b, _ = _lib.zolotarev(20, 1e-3, 8.0)
    lam, U = np.linalg.eigh(H)
    rfun = sum(ak / (lam * lam + bk) for ak, bk in zip(a, b))
    exact = U @ (lam * lam * rfun * rfun * (U.conj().T @ x))
    al, rho, rs = _krylov(H, x, tol)
    N = len(al)
    be = rho[1:] / rho[:-1]
    diag = 1 / al + np.concatenate([[0.0], be[:N - 1] / al[:N - 1]])
    off = np.sqrt(be[:N - 1]) / al[:N - 1]
    T = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    e1 = np.zeros(N)
    e1[0] = 1
    g = sum(ak * np.linalg.solve(T + bk * np.eye(N), e1) for ak, bk in zip(a, b))
    h = sum(ak * np.linalg.solve(T + bk * np.eye(N), g) for ak, bk in zip(a, b))
    c2 = np.sqrt(rho[0]) * (-1.0) ** np.arange(N) * h / np.sqrt(rho[:N])
    r2x = sum(c2[j] * rs[j] for j in range(N))          # r(A)^2 x on the residuals
    got = H @ (H @ r2x)                                   # eps^2 x = A r(A)^2 x
    err = np.linalg.norm(got - exact) / np.linalg.norm(x)
    assert err < 20 * tol
    # and eps^2 x differs from x by the rational error only (|eps^2 - 1| <= 2 delta)
    assert np.linalg.norm(exact - x) / np.linalg.norm(x) < 1e-7
