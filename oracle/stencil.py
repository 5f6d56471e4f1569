"""Semi-discrete Hamiltonian and boundary sets (paper Sec. 2).

Test infrastructure: part of the FP64 oracle, not of the product path.

Conventions
-----------
* A wavefunction on the box is an array ``psi[z, y, x]`` (x fastest); a batch
  carries a trailing orbital axis ``psi[z, y, x, j]``.
* ``R`` is the half-width of the finite-difference stencil; the 1D second
  derivative is ``sum_{k=-R..R} c_k u_{j+k} / h^2`` with ``c_{-k} = c_k``
  (Sec. 2 prints the R = 2 weights; App. D prints R = 4).
* The box Hamiltonian is H_{I,I} = -(1/2) Delta_h + V with the values outside
  the box treated as absent (zero), i.e. the I,I block of the full-lattice
  Hamiltonian (Sec. 2, block system).
"""
from __future__ import annotations

from fractions import Fraction
from typing import Dict, List, Tuple

import numpy as np


# ---------------------------------------------------------------------------
# Finite-difference weights
# ---------------------------------------------------------------------------

def fd_weights_exact(R: int) -> List[Fraction]:
    """Central second-derivative weights c_0..c_R of half-width R.

    They are the unique symmetric weights exact on polynomials of degree
    2R+1: with c_{-k} = c_k the conditions are c_0 + 2 sum_k c_k = 0,
    2 sum_k c_k k^2 = 2 and sum_k c_k k^{2m} = 0 for m = 2..R.  Solved here in
    exact rational arithmetic (plain Gaussian elimination on Fractions).
    The paper prints R = 2 (Sec. 2 and App. B) and R = 4 (App. D, where the
    printed centre weight has a sign typo: it must be -205/72 so the weights
    sum to zero).
    """
    if R < 1:
        raise ValueError("R >= 1")
    n = R + 1  # unknowns c_0..c_R
    A = [[Fraction(0)] * n for _ in range(n)]
    b = [Fraction(0)] * n
    for m in range(n):
        for k in range(n):
            if k == 0:
                A[m][k] = Fraction(1 if m == 0 else 0)
            else:
                A[m][k] = Fraction(2 * k ** (2 * m))
        b[m] = Fraction(2 if m == 1 else 0)
    # Gaussian elimination with exact pivots
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col] / A[col][col]
                A[r] = [a - f * p for a, p in zip(A[r], A[col])]
                b[r] -= f * b[col]
    return [b[i] / A[i][i] for i in range(n)]


def fd_weights(R: int) -> np.ndarray:
    """float64 copy of :func:`fd_weights_exact`."""
    return np.array([float(c) for c in fd_weights_exact(R)], dtype=np.float64)


# ---------------------------------------------------------------------------
# Box Hamiltonian H_{I,I}
# ---------------------------------------------------------------------------

def _shifted(a: np.ndarray, axis: int, k: int, periodic: bool) -> np.ndarray:
    """Array b with b[i] = a[i + k] along ``axis``; zero (or wrapped) outside."""
    if periodic:
        return np.roll(a, -k, axis=axis)
    out = np.zeros_like(a)
    n = a.shape[axis]
    if abs(k) >= n:
        return out
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    if k >= 0:
        src[axis] = slice(k, n)
        dst[axis] = slice(0, n - k)
    else:
        src[axis] = slice(0, n + k)
        dst[axis] = slice(-k, n)
    out[tuple(dst)] = a[tuple(src)]
    return out


def laplacian(psi: np.ndarray, h: float, R: int, periodic: bool = False) -> np.ndarray:
    """Delta_h psi = sum over the three axes of sum_k c_k psi(p + k e_a) / h^2.

    The three spatial axes are the first three array axes; values outside the
    box are zero (the I,I block) unless ``periodic``.
    """
    c = fd_weights(R)
    out = np.zeros_like(psi)
    for axis in range(3):
        out += c[0] * psi
        for k in range(1, R + 1):
            out += c[k] * (_shifted(psi, axis, k, periodic) + _shifted(psi, axis, -k, periodic))
    return out / (h * h)


def apply_H(psi: np.ndarray, V: np.ndarray, h: float, R: int, periodic: bool = False) -> np.ndarray:
    """H_{I,I} psi = -(1/2) Delta_h psi + V psi (hbar = m = 1, Sec. 2)."""
    if psi.ndim == 4:
        Vb = V[..., None]
    else:
        Vb = V
    return -0.5 * laplacian(psi, h, R, periodic) + Vb * psi


def dense_H(shape, V, h, R, periodic=False) -> np.ndarray:
    """Dense H_{I,I} (small boxes only) assembled column by column."""
    n = int(np.prod(shape))
    Hm = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        Hm[:, j] = apply_H(e.reshape(shape), V, h, R, periodic).ravel()
    return Hm


# ---------------------------------------------------------------------------
# Boundary sets (Sec. 2 definition of Gamma; App. A definition of Sigma)
# ---------------------------------------------------------------------------

def gamma_mask(shape, R: int) -> np.ndarray:
    """Box points coupled by the stencil to at least one exterior point:
    some coordinate within R of a face."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    m = np.zeros(shape, dtype=bool)
    for c, n in ((z, nz), (y, ny), (x, nx)):
        m |= (c < R) | (c > n - 1 - R)
    return m


def gamma_points(shape, R: int) -> np.ndarray:
    """Gamma as an (n_Gamma, 3) array of (z, y, x) indices in C order; this
    fixes the ordering of every box-form boundary vector."""
    return np.argwhere(gamma_mask(shape, R))


def sigma_points(shape, R: int) -> np.ndarray:
    """Sigma (App. A): exterior points coupled to the box.  With an
    axis-aligned stencil these are the points with exactly one coordinate out
    of range, by at most R.  Returned as (n_Sigma, 3) (z, y, x) indices,
    possibly negative or >= n."""
    pts = []
    dims = tuple(shape)
    for axis in range(3):
        n = dims[axis]
        others = [a for a in range(3) if a != axis]
        outside = list(range(-R, 0)) + list(range(n, n + R))
        for o in outside:
            for i in range(dims[others[0]]):
                for j in range(dims[others[1]]):
                    p = [0, 0, 0]
                    p[axis] = o
                    p[others[0]] = i
                    p[others[1]] = j
                    pts.append(tuple(p))
    return np.array(sorted(pts), dtype=np.int64)


def coupling_gamma_sigma(gamma: np.ndarray, sigma: np.ndarray, h: float, R: int) -> np.ndarray:
    """H_{Gamma,Sigma}: entry -c_{|p-q|}/(2h^2) when p and q lie on one axis line
    within R of each other (the off-diagonal block of -Delta_h/2)."""
    c = fd_weights(R)
    Hgs = np.zeros((len(gamma), len(sigma)), dtype=np.float64)
    sig_index: Dict[Tuple[int, int, int], int] = {tuple(q): j for j, q in enumerate(sigma)}
    for i, p in enumerate(gamma):
        for axis in range(3):
            for k in range(-R, R + 1):
                if k == 0:
                    continue
                q = list(p)
                q[axis] += k
                j = sig_index.get(tuple(q))
                if j is not None:
                    Hgs[i, j] = -c[abs(k)] / (2.0 * h * h)
    return Hgs


def n_gamma(n: int, R: int) -> int:
    """|Gamma| for a cube of n points per axis."""
    return n ** 3 - max(n - 2 * R, 0) ** 3
