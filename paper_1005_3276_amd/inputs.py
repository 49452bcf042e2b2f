"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds random-number generation only -- none of the method's arithmetic -- so
that the GPU path and the CPU oracle receive bit-identical inputs.

Distributions (workload recipe):
  * background scalar phi_x ~ CN(0, sigma2): real and imaginary parts i.i.d.
    N(0, sigma2/2), one complex number per site, shape (T, Z, Y, X);
  * sources / pseudofermion noise ~ CN(0, 1) per spinor component, shape
    (nrhs, T, Z, Y, X, 4).
Generator: numpy PCG64 with the given seed; phi is drawn first, then sources.
"""
import numpy as np

BASE_SEED = 10053276


def config_seed(config_index: int) -> int:
    return BASE_SEED * 10 + config_index


def draw(dims, nrhs=1, sigma2=0.25, seed=0):
    """Return (phi, src): phi complex128 (T,Z,Y,X); src complex128 (nrhs,T,Z,Y,X,4)."""
    X, Y, Z, T = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.standard_normal((2, T, Z, Y, X))
    phi = np.sqrt(sigma2 / 2.0) * (u[0] + 1j * u[1])
    v = rng.standard_normal((2, nrhs, T, Z, Y, X, 4))
    src = np.sqrt(0.5) * (v[0] + 1j * v[1])
    return phi.astype(np.complex128), src.astype(np.complex128)


def gaussian_field(dims, nrhs=1, seed=0):
    """CN(0,1) spinor field(s) only, shape (nrhs, T, Z, Y, X, 4)."""
    X, Y, Z, T = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal((2, nrhs, T, Z, Y, X, 4))
    return (np.sqrt(0.5) * (v[0] + 1j * v[1])).astype(np.complex128)
