"""Long-range TDHF potentials (Sec. 4.3): the Yukawa and Coulomb fields of the
density, from the Helmholtz and Poisson problems

    (Delta_h - 1/a^2) W_Y = -4 pi V0 a rho,      Delta_h W_C = -2 pi e^2 rho,

on the box, with Delta_h the wavefunctions' finite-difference Laplacian of
half-width R and zero values outside the box (the paper solves both "with the
same discretization as the wave functions"; the boundary values are not
stated, and zero outside the box is the reading taken).

Test infrastructure: part of the FP64 oracle, not of the product path.  The
systems are solved exactly (sparse LU); the device solves them by
conjugate gradients.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import erfc

from .stencil import fd_weights


def neg_laplacian(shape, h: float, R: int) -> sp.csr_matrix:
    """-Delta_h on the box in C order of (z, y, x), zero outside (SPD)."""
    nz, ny, nx = shape
    c = fd_weights(R)
    n = nz * ny * nx
    idx = np.arange(n).reshape(shape)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.full(n, -3.0 * c[0] / (h * h))]
    for axis in range(3):
        for k in range(1, R + 1):
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[axis] = slice(0, shape[axis] - k)
            hi[axis] = slice(k, shape[axis])
            a, b = idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()
            w = np.full(a.size, -c[k] / (h * h))
            rows += [a, b]
            cols += [b, a]
            vals += [w, w]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def _solve(rho, h, R, mu2, scale):
    A = neg_laplacian(rho.shape, h, R)
    if mu2:
        A = A + mu2 * sp.identity(A.shape[0], format="csr")
    return spla.spsolve(A.tocsc(), scale * rho.ravel()).reshape(rho.shape)


def yukawa(rho: np.ndarray, h: float, R: int, v0: float, a: float) -> np.ndarray:
    """W_Y: (-Delta_h + 1/a^2) W_Y = 4 pi V0 a rho."""
    return _solve(rho, h, R, 1.0 / (a * a), 4.0 * math.pi * v0 * a)


def coulomb(rho: np.ndarray, h: float, R: int, e2: float) -> np.ndarray:
    """W_C: -Delta_h W_C = 2 pi e^2 rho."""
    return _solve(rho, h, R, 0.0, 2.0 * math.pi * e2)


def yukawa_gaussian(r: np.ndarray, q: float, sigma: float, v0: float, a: float) -> np.ndarray:
    """Continuum W_Y = V0 int exp(-|r - r'|/a) / (|r - r'|/a) rho(r') dr' for
    rho = q (2 pi sigma^2)^(-3/2) exp(-r^2 / (2 sigma^2)): the screened
    potential of a Gaussian charge,
    (q a V0 / 2r) e^{sigma^2/2a^2} [e^{-r/a} erfc((sigma^2/a - r)/(sqrt2 sigma))
                                   - e^{r/a} erfc((sigma^2/a + r)/(sqrt2 sigma))]."""
    r = np.asarray(r, dtype=np.float64)
    s2 = math.sqrt(2.0) * sigma
    pre = q * a * v0 / (2.0 * r) * math.exp(sigma * sigma / (2.0 * a * a))
    return pre * (np.exp(-r / a) * erfc((sigma * sigma / a - r) / s2) - np.exp(r / a) * erfc((sigma * sigma / a + r) / s2))
