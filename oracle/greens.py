"""Lattice Green's functions and the half-line DtN symbol.

Test infrastructure: part of the FP64 oracle, not of the product path.

* :func:`gf3d_table` -- the free-space lattice Green's function
  G~(s) = (H - i s I)^{-1} on Z^3 for H = -(1/2) Delta_h, written as the
  Brillouin-zone Fourier integral of App. D and evaluated by the trapezoidal
  rule on an L-periodic lattice (an inverse FFT).  The periodic images decay
  like exp(-Re sqrt(-2is) r), so a lattice a few decay lengths larger than
  the box reproduces the Z^3 function to rounding.
* :func:`gf1d_appendix_b` -- App. B's closed form for the 1D five-point
  stencil (roots of the characteristic quartic).  The printed formula has a
  sign error in the second coefficient: the function that solves the 1D
  equation is b1 u1^|j| - b2 u3^|j|.
* :func:`halfline_symbol` -- the DtN map of the half-space exterior of one
  face, per transverse Fourier mode: an R x R matrix k^(theta; s).  It is the
  1D version of the Sec. 2 construction: the exterior solution is a
  combination of the decaying characteristic modes of the 1D recurrence (the
  App. B construction generalised to any R), matched to the R boundary
  layers, and then mapped to f_Gamma by the coupling block.
"""
from __future__ import annotations

import cmath
import math

import numpy as np

from .stencil import fd_weights


def symbol_1d(theta: np.ndarray, h: float, R: int) -> np.ndarray:
    """Fourier symbol of -(1/2) d^2/dx^2 discretised with half-width R:
    (1/(2h^2)) (-c_0 - 2 sum_k c_k cos k theta)  (>= 0)."""
    c = fd_weights(R)
    acc = -c[0] * np.ones_like(theta)
    for k in range(1, R + 1):
        acc = acc - 2.0 * c[k] * np.cos(k * theta)
    return acc / (2.0 * h * h)


def default_lattice(n_max: int, R: int, s: float, h: float) -> int:
    """Periodic lattice size for the 3D Green's function table: at least
    2(n + 2R) + 35/(sqrt(s) h) points, rounded up to a power of two."""
    need = 2 * (n_max + 2 * R) + int(math.ceil(35.0 / (math.sqrt(s) * h)))
    L = 16
    while L < need:
        L *= 2
    return L


def gf3d_table(s: float, h: float, R: int, L: int) -> np.ndarray:
    """G~(Delta) for Delta in Z_L^3 (index Delta mod L), complex128 (L, L, L).

    Trapezoidal rule for G~(Delta) = (2 pi)^{-3} int exp(i theta.Delta) /
    (sigma(theta) - i s) d theta  (App. D with H~ = H - i s I).
    """
    th = 2.0 * np.pi * np.arange(L) / L
    s1 = symbol_1d(th, h, R)
    sig = s1[:, None, None] + s1[None, :, None] + s1[None, None, :]
    ghat = 1.0 / (sig - 1j * s)
    return np.fft.ifftn(ghat)


def gf1d_table(shift: complex, h: float, R: int, L: int) -> np.ndarray:
    """1D lattice Green's function of (-(1/2) d^2_h + shift) on Z, by the same
    periodic trapezoidal rule; index j mod L."""
    th = 2.0 * np.pi * np.arange(L) / L
    return np.fft.ifft(1.0 / (symbol_1d(th, h, R) + shift))


def gf1d_appendix_b(s: float, h: float, j: np.ndarray) -> np.ndarray:
    """App. B closed form for the five-point stencil (R = 2).

    Returns G_j solving 2 i s G_j + sum_k c_k G_{j+k} / h^2 = delta_j
    (App. B's discrete equation with a unit source), i.e.
    G = -(1/2) (H - i s)^{-1}.  Roots u1, u3 of the characteristic quartic
    are the two inside the unit circle; the second coefficient enters with a
    minus sign (the printed plus sign does not satisfy the equation).
    """
    a = cmath.sqrt(9 + 6j * s * h * h)
    u1 = 4 + a - cmath.sqrt(6j * s * h * h + 8 * a + 24)
    u3 = 4 - a - cmath.sqrt(6j * s * h * h - 8 * a + 24)
    b1 = (h * h / 2) * cmath.sqrt(3 / ((3 + 2j * s * h * h) * (24 + 6j * s * h * h + 8 * a)))
    b2 = (h * h / 2) * cmath.sqrt(3 / ((3 + 2j * s * h * h) * (24 + 6j * s * h * h - 8 * a)))
    j = np.abs(np.asarray(j))
    return b1 * u1 ** j - b2 * u3 ** j


def transverse_shift(theta1: np.ndarray, theta2: np.ndarray, h: float, R: int) -> np.ndarray:
    """tau(theta) = symbol of -(1/2) Delta_h in the two directions parallel to
    a face, for transverse Fourier angles (theta1, theta2)."""
    return symbol_1d(theta1, h, R) + symbol_1d(theta2, h, R)


def coupling_1d(h: float, R: int) -> np.ndarray:
    """1D H_{Gamma,Sigma} for one face: rows = layers p = 0..R-1 (distance from
    the face), columns = exterior points q = -1..-R (q = -1 first).  Entry
    -c_{p-q}/(2h^2) when p - q <= R."""
    c = fd_weights(R)
    Hgs = np.zeros((R, R))
    for p in range(R):
        for qi in range(R):
            q = -1 - qi
            if p - q <= R:
                Hgs[p, qi] = -c[p - q] / (2.0 * h * h)
    return Hgs


def halfline_symbol(shift: np.ndarray, h: float, R: int) -> np.ndarray:
    """Half-line DtN symbol for shift = tau(theta) - i s.

    The exterior is x <= -1 on the line through a face point; the layers
    0..R-1 form Gamma.  The exterior field solves (H_1D + shift) Phi = 0 at
    every exterior row, decays as x -> -inf and equals the data on Gamma.  The
    characteristic polynomial u^R [(-(1/2h^2)) sum_k c_|k| u^k + shift] has R
    roots inside the unit circle; Phi(x) = sum_j beta_j u_j^{(R-1)-x} spans
    the decaying solutions.  Matching the R data values fixes beta, and
    f_Gamma = H_{Gamma,Sigma} Phi_Sigma gives k^ = H_gs W V^{-1}.

    ``shift`` may be an array; the result has shape shift.shape + (R, R).
    """
    shift = np.asarray(shift, dtype=np.complex128)
    c = fd_weights(R)
    flat = shift.ravel()
    m = flat.size
    deg = 2 * R
    # polynomial coefficients, highest power first: power k+R for k = R..-R
    coeffs = np.zeros((m, deg + 1), dtype=np.complex128)
    for k in range(-R, R + 1):
        coeffs[:, R - k] += -c[abs(k)] / (2.0 * h * h)
    coeffs[:, R] += flat
    # companion matrices (monic)
    lead = coeffs[:, 0]
    comp = np.zeros((m, deg, deg), dtype=np.complex128)
    comp[:, 0, :] = -coeffs[:, 1:] / lead[:, None]
    for i in range(1, deg):
        comp[:, i, i - 1] = 1.0
    roots = np.linalg.eigvals(comp)
    order = np.argsort(np.abs(roots), axis=1)
    inner = np.take_along_axis(roots, order[:, :R], axis=1)  # |u| < 1
    p = np.arange(R)
    q = -1 - np.arange(R)
    V = inner[:, None, :] ** ((R - 1) - p)[None, :, None]       # (m, R, R) rows p
    W = inner[:, None, :] ** ((R - 1) - q)[None, :, None]       # rows q
    Hgs = coupling_1d(h, R)
    # k^ = Hgs W V^{-1}
    WVinv = np.linalg.solve(np.transpose(V, (0, 2, 1)), np.transpose(W, (0, 2, 1)))
    WVinv = np.transpose(WVinv, (0, 2, 1))
    K = np.einsum("pq,mqr->mpr", Hgs, WVinv)
    return K.reshape(shift.shape + (R, R))


def halfline_symbol_bruteforce(shift: complex, h: float, R: int, length: int = 4000) -> np.ndarray:
    """The same R x R symbol from a direct sparse solve on a long truncated
    exterior line (x = -length..-1, zero beyond): -H_{Gamma,II}
    (H_{II,II} + shift)^{-1} H_{II,Gamma}.  Used only to pin
    :func:`halfline_symbol`."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    c = fd_weights(R)
    n = length
    diags = []
    offs = []
    for k in range(-R, R + 1):
        diags.append(np.full(n - abs(k), -c[abs(k)] / (2.0 * h * h), dtype=np.complex128))
        offs.append(k)
    Hii = sp.diags(diags, offs, shape=(n, n), format="csc").astype(np.complex128)
    Hii = Hii + shift * sp.identity(n, format="csc")
    # exterior index e corresponds to x = -n + e (e = n-1 is x = -1)
    Hig = np.zeros((n, R), dtype=np.complex128)
    for e in range(n - R, n):
        x = -n + e
        for p in range(R):
            if p - x <= R:
                Hig[e, p] = -c[p - x] / (2.0 * h * h)
    sol = spla.spsolve(Hii, Hig)
    return -(Hig.T @ sol)
