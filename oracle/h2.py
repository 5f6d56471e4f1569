"""H2 objective of the first-order interpolation point (face form, R = 1).

Test infrastructure: part of the FP64 oracle, not of the product path.

The paper closes (Sec. 5, summary and discussions) by proposing to choose the
first-order interpolation point as the minimiser of ||K(s) - R11(s)||_H2.
For the face form this is evaluated per half-space and per transverse
Fourier mode theta = (theta1, theta2):

    J(s1) = P^-2 sum_theta (1/2pi) int_R |k^(theta; i w) - r(theta; i w)|^2 dw,

with k^ the exact half-line DtN symbol on the imaginary axis (the limit from
Re s > 0) and r(theta; s) = a / (s - b_w(theta)) the symbol of the operator
that is actually applied: a = -i H_gs H_gs^T and b_w the Fourier series of
the (windowed, truncated) kernel of B built at s1 (Theorem 3.2 per mode).

Readings (not fixed by the paper, stated here and used identically by the
HIP path):
* modes: the P x P grid theta_j = 2 pi j / P;
* frequencies: w = W0 + W0 tan(phi), phi on N midpoints of (-pi/2, pi/2),
  W0 = -3/h^2 (the centre of the exterior spectrum [-6/h^2, 0] of -Delta_h/2
  reflected onto the imaginary axis), weights W0 sec^2(phi) pi/N in
  magnitude;
* on the axis, b = 1 + h^2 (tau + w) is real; the decaying root of
  u^2 - 2 b u + 1 = 0 is 1/(b + sqrt(b^2 - 1)) for b > 1,
  1/(b - sqrt(b^2 - 1)) for b < -1, and b + i sqrt(1 - b^2) on the cut
  (the limit of the |u| < 1 root as Re s -> 0+), and k^ = -u / (2 h^2).
"""
from __future__ import annotations

import math

import numpy as np

from . import dtn, greens


def halfline_symbol_axis(tau, omega, h: float):
    """k^(theta; i omega) for R = 1 as the limit from Re s > 0."""
    b = 1.0 + h * h * (np.asarray(tau, dtype=np.float64) + np.asarray(omega, dtype=np.float64))
    b = np.asarray(b, dtype=np.float64)
    u = np.empty(b.shape, dtype=np.complex128)
    hi = b > 1.0
    lo = b < -1.0
    mid = ~(hi | lo)
    u[hi] = 1.0 / (b[hi] + np.sqrt(b[hi] * b[hi] - 1.0))
    u[lo] = 1.0 / (b[lo] - np.sqrt(b[lo] * b[lo] - 1.0))
    u[mid] = b[mid] + 1j * np.sqrt(1.0 - b[mid] * b[mid])
    return -u / (2.0 * h * h)


def frequency_nodes(h: float, N: int):
    """(omega, weight) of the tan-mapped midpoint rule on the real line."""
    w0 = 3.0 / (h * h)
    phi = -0.5 * math.pi + (np.arange(N) + 0.5) * math.pi / N
    omega = -w0 + w0 * np.tan(phi)
    weight = w0 / np.cos(phi) ** 2 * (math.pi / N)
    return omega, weight


def kernel_symbol(ker: np.ndarray, P: int) -> np.ndarray:
    """Symbol b_w(theta) = sum_p k(p) exp(-i p.theta) of an R = 1 face kernel
    (index p + w) on the P x P mode grid (the inverse of
    :func:`dtn.face_kernel_from_symbol`)."""
    k = ker[0, 0]
    w = (k.shape[0] - 1) // 2
    th = dtn.symbol_grid(P)
    p = np.arange(-w, w + 1)
    e = np.exp(-1j * np.outer(th, p))          # (P, 2w+1)
    return e @ k @ e.T                          # (P, P)


def h2_objective(h: float, s1: float, w: int, P: int = 64, N: int = 4096, window: bool = True) -> float:
    """J(s1) as defined in the module docstring (first order, R = 1)."""
    fo = dtn.face_first(h, 1, s1, w, window=window)
    a = fo.a[0, 0]
    bw = kernel_symbol(fo.kernel, P)
    th = dtn.symbol_grid(P)
    tau = greens.transverse_shift(th[:, None], th[None, :], h, 1)
    omega, weight = frequency_nodes(h, N)
    total = 0.0
    for i in range(P):
        k = halfline_symbol_axis(tau[i][:, None], omega[None, :], h)          # (P, N)
        r = a / (1j * omega[None, :] - bw[i][:, None])
        total += float(np.sum(np.abs(k - r) ** 2 * weight[None, :]))
    return total / (2.0 * math.pi * P * P)


def one_pole_h2(a: complex, b: complex) -> float:
    """(1/2pi) int |a / (i w - b)|^2 dw = |a|^2 / (2 |Re b|) for Re b < 0, the
    closed form that pins the frequency rule."""
    return abs(a) ** 2 / (-2.0 * b.real)
