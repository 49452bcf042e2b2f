"""Rational approximations of powers for the RHMC layers of Sec. 7.3.

The pseudofermion heatbath applies (M^dag M)^{1/8} and the action (M^dag M)^{-1/4}
through partial fractions

    x^alpha ~ a0 + sum_i alpha_i / (x + beta_i),   beta_i > 0,

on the spectral interval [lo, hi] of M^dag M (the paper uses degree 20).  The
coefficients are set-up data for ``Lattice.rational`` / ``ov_rational``; this
module computes them on the host.

Method (near-minimax in relative error): the shifts beta_i start from the
Zolotarev shifts of 1/sqrt(x) on the same interval (optimal for alpha = -1/2)
and are then moved by a variable-projection least-squares fit (Golub-Pereyra:
for fixed shifts the residues are a linear least-squares problem) under
Lawson's iteratively reweighted weights, which drive the weighted
least-squares solution towards the minimax one.  For 0 < alpha < 1 the fit is
done for x^(alpha - 1) without constant and multiplied by x:
x sum c_i/(x + p_i) = sum c_i - sum c_i p_i/(x + p_i).
"""
import functools

import numpy as np


def _fit(expo, lo, hi, shifts0, const, samples, rounds, lawson):
    from scipy.optimize import least_squares

    x = np.exp(np.linspace(np.log(lo), np.log(hi), samples))
    f = x ** expo

    def design(logp):
        cols = ([np.ones_like(x)] if const else []) + [1.0 / (x + b) for b in np.exp(logp)]
        return np.column_stack(cols) / f[:, None]

    w = np.full_like(x, 1.0 / samples)
    logp = np.log(shifts0)
    best = None
    for _ in range(rounds):
        sw = np.sqrt(w)

        def resid(lp):
            A = design(lp)
            c, *_ = np.linalg.lstsq(A * sw[:, None], sw, rcond=None)
            return (A @ c - 1.0) * sw

        logp = least_squares(resid, logp, method="lm", max_nfev=4000).x
        A = design(logp)
        for _ in range(lawson):
            sw = np.sqrt(w)
            c, *_ = np.linalg.lstsq(A * sw[:, None], sw, rcond=None)
            e = A @ c - 1.0
            w = w * np.abs(e) + 1e-300
            w /= w.sum()
        err = np.abs(e).max()
        if best is None or err < best[0]:
            best = (err, np.exp(logp).copy(), c.copy())
    return best


def power_approx(alpha, lo, hi, n=20, samples=1500, rounds=2, lawson=20):
    """Coefficients (a0, alphas, betas, max_rel_err) of x^alpha on [lo, hi].

    -1 < alpha < 1, alpha != 0; 0 < lo < hi.  max_rel_err is the largest
    |r(x)/x^alpha - 1| on a log-spaced sample of the interval.  Results are
    cached per argument set.
    """
    if not (-1.0 < alpha < 1.0) or alpha == 0.0 or not (0.0 < lo < hi):
        raise ValueError("need -1 < alpha < 1, alpha != 0 and 0 < lo < hi")
    a0, al, be, err = _power_approx(float(alpha), float(lo), float(hi), int(n), int(samples),
                                    int(rounds), int(lawson))
    return a0, al.copy(), be.copy(), err


@functools.lru_cache(maxsize=32)
def _power_approx(alpha, lo, hi, n, samples, rounds, lawson):
    from . import _lib

    _, z_shifts, _ = _lib.zolotarev(n, np.sqrt(lo), np.sqrt(hi))
    if alpha < 0:
        err, p, c = _fit(alpha, lo, hi, z_shifts, True, samples, rounds, lawson)
        a0, res = float(c[0]), c[1:]
    else:
        err, p, c = _fit(alpha - 1.0, lo, hi, z_shifts, False, samples, rounds, lawson)
        a0, res = float(np.sum(c)), -c * p
    order = np.argsort(p)
    return a0, np.asarray(res)[order], np.asarray(p)[order], float(err)


def evaluate(x, a0, alphas, betas):
    """r(x) = a0 + sum_i alphas_i / (x + betas_i) for an array x."""
    x = np.asarray(x, dtype=np.float64)
    return a0 + sum(a / (x + b) for a, b in zip(alphas, betas))
