"""Discrete DtN map and its rational approximations.

Test infrastructure: part of the FP64 oracle, not of the product path.

Box form (the paper's own construction)
    K(s) = -(I - H_{Gamma,Sigma} G~_{Sigma,Gamma})^{-1}
             H_{Gamma,Sigma} G~_{Sigma,Sigma} H_{Sigma,Gamma}
    (App. A, discrete boundary-element formula), dense n_Gamma x n_Gamma.
    Zeroth order (Sec. 3, zeroth-order approximation): M = K(s0).
    First order (Sec. 3, first-order stability theorem):
        A = -i H_{Gamma,II} H_{II,Gamma},  B = s1 I - A K(s1)^{-1}.
    First order from two finite points (the variant used in the experiments,
    Sec. 4.2/4.3): R11(s1) = K(s1), R11(s2) = K(s2), which gives
        B = (s2 K2 - s1 K1)(K2 - K1)^{-1},  A = (s1 I - B) K1.

Face form (a construction for large boxes; not in the paper)
    The exterior of the box is replaced by the six half-spaces beyond its
    faces.  Each is translation invariant along its face, so its DtN map is a
    convolution along the face whose Fourier symbol, per transverse mode, is
    the half-line symbol k^(theta; s) (R x R, layers).  The coupling
    H_{Gamma,Sigma} of each face, hence A and Q of the first-order theorem,
    are exactly the paper's.  Operators are the Toeplitz sections over each
    face's R x n1 x n2 slab of the kernels
        k_f(p) = (2pi)^{-2} int k^(theta) exp(i p.theta) d theta
    truncated to |p|_inf <= w and multiplied by the separable triangular
    (Fejer) window (1 - |p1|/(w+1))(1 - |p2|/(w+1)).  The window's Fourier
    series is a non-negative kernel of unit mass, so the smoothed symbol keeps
    the sign conditions of the two stability theorems mode by mode, and a
    Toeplitz section of a sign-definite symbol is sign-definite.  With
    ``window=None`` the full section (no window, |p| < n) is used.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

from . import greens
from .stencil import coupling_gamma_sigma, gamma_points, sigma_points


# ---------------------------------------------------------------------------
# Box form
# ---------------------------------------------------------------------------

def dtn_box(shape, h: float, R: int, s: float, L: Optional[int] = None) -> np.ndarray:
    """K(s) for the box ``shape`` by the App. A formula (dense, complex128)."""
    gamma = gamma_points(shape, R)
    sigma = sigma_points(shape, R)
    Hgs = coupling_gamma_sigma(gamma, sigma, h, R)
    if L is None:
        L = greens.default_lattice(max(shape), R, s, h)
    G = greens.gf3d_table(s, h, R, L)

    def gather(P, Q):
        out = np.empty((len(P), len(Q)), dtype=np.complex128)
        for i0 in range(0, len(P), 512):
            d = (P[i0:i0 + 512, None, :] - Q[None, :, :]) % L
            out[i0:i0 + 512] = G[d[..., 0], d[..., 1], d[..., 2]]
        return out

    Gsg = gather(sigma, gamma)
    Gss = gather(sigma, sigma)
    T = Hgs @ Gsg
    S = Hgs @ Gss @ Hgs.T
    n = len(gamma)
    return -np.linalg.solve(np.eye(n) - T, S)


def dtn_box_bruteforce(shape, h: float, R: int, s: float, pad: int) -> np.ndarray:
    """K(s) = -H_{Gamma,II} (H_{II,II} - i s)^{-1} H_{II,Gamma} (Sec. 2) with the
    exterior truncated to ``pad`` layers around the box (zero beyond).  A
    direct sparse solve, used only to pin :func:`dtn_box` on tiny boxes."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from .stencil import fd_weights
    nz, ny, nx = shape
    big = (nz + 2 * pad, ny + 2 * pad, nx + 2 * pad)
    inside = np.zeros(big, dtype=bool)
    inside[pad:pad + nz, pad:pad + ny, pad:pad + nx] = True
    ext_idx = -np.ones(big, dtype=np.int64)
    ext_pts = np.argwhere(~inside)
    ext_idx[tuple(ext_pts.T)] = np.arange(len(ext_pts))
    c = fd_weights(R)
    rows, cols, vals = [], [], []
    for e, p in enumerate(ext_pts):
        rows.append(e); cols.append(e); vals.append(-3 * c[0] / (2 * h * h) - 1j * s)
        for axis in range(3):
            for k in range(1, R + 1):
                for sgn in (1, -1):
                    q = p.copy(); q[axis] += sgn * k
                    if np.all(q >= 0) and np.all(q < big):
                        j = ext_idx[tuple(q)]
                        if j >= 0:
                            rows.append(e); cols.append(j); vals.append(-c[k] / (2 * h * h))
    Hii = sp.csc_matrix((vals, (rows, cols)), shape=(len(ext_pts), len(ext_pts)))
    gamma = gamma_points(shape, R)
    Hig = np.zeros((len(ext_pts), len(gamma)), dtype=np.complex128)
    for g, p in enumerate(gamma):
        pb = p + pad
        for axis in range(3):
            for k in range(1, R + 1):
                for sgn in (1, -1):
                    q = pb.copy(); q[axis] += sgn * k
                    if np.all(q >= 0) and np.all(q < big):
                        j = ext_idx[tuple(q)]
                        if j >= 0:
                            Hig[j, g] = -c[k] / (2 * h * h)
    sol = spla.spsolve(Hii, Hig)
    return -(Hig.T @ sol)


@dataclasses.dataclass
class BoxOperators:
    order: str
    gamma: np.ndarray                   # (n_Gamma, 3) z,y,x
    M: Optional[np.ndarray] = None      # zeroth order
    A: Optional[np.ndarray] = None      # first order
    B: Optional[np.ndarray] = None
    Q: Optional[np.ndarray] = None      # Lyapunov weight (Theorem-based first order)
    # second order (Sec. 3.3): R22(s) = (s^2 I - s B1 - B0)^{-1} (s A1 + A0), C = B1 A1 + A0
    B1: Optional[np.ndarray] = None
    B0: Optional[np.ndarray] = None
    A1: Optional[np.ndarray] = None
    A0: Optional[np.ndarray] = None
    C: Optional[np.ndarray] = None


def box_coupling_product(shape, h, R) -> np.ndarray:
    """H_{Gamma,II} H_{II,Gamma} = H_{Gamma,Sigma} H_{Sigma,Gamma} (real symmetric)."""
    gamma = gamma_points(shape, R)
    sigma = sigma_points(shape, R)
    Hgs = coupling_gamma_sigma(gamma, sigma, h, R)
    return Hgs @ Hgs.T


def box_zeroth(shape, h, R, s0, L=None) -> BoxOperators:
    return BoxOperators("zeroth", gamma_points(shape, R), M=dtn_box(shape, h, R, s0, L))


def box_first(shape, h, R, s1, s2=math.inf, L=None) -> BoxOperators:
    """First-order coefficients.  s2 = inf: the stability theorem's pair
    (derivative matching at lambda = 1/s -> 0 plus R11(s1) = K(s1)); finite
    s2: two-point interpolation."""
    gamma = gamma_points(shape, R)
    HH = box_coupling_product(shape, h, R)
    K1 = dtn_box(shape, h, R, s1, L)
    n = len(gamma)
    if math.isinf(s2):
        A = -1j * HH
        # A K1^{-1}: K1 and A are complex symmetric, so A K1^{-1} = (K1^{-1} A)^T
        AK1inv = np.linalg.solve(K1, A).T
        B = s1 * np.eye(n) - AK1inv
        Q = np.linalg.inv(HH)
        return BoxOperators("first", gamma, A=A, B=B, Q=Q)
    K2 = dtn_box(shape, h, R, s2, L)
    # B (K2 - K1) = s2 K2 - s1 K1  ->  (K2 - K1)^T B^T = (s2 K2 - s1 K1)^T
    B = np.linalg.solve((K2 - K1).T, (s2 * K2 - s1 * K1).T).T
    A = (s1 * np.eye(n) - B) @ K1
    return BoxOperators("first", gamma, A=A, B=B, Q=None)


def interp_second(Ks, s_pts):
    """Coefficients of the second-order rational approximation (Sec. 3.3),
    R22(s) = (s^2 I - s B1 - B0)^{-1} (s A1 + A0), from R22(s_j) = K(s_j) at
    four points: (s_j^2 I - s_j B1 - B0) K_j = s_j A1 + A0, i.e.
    [B1 B0 A1 A0] [s_j K_j; K_j; s_j I; I] = s_j^2 K_j for j = 1..4, solved as
    one linear system.  Works on dense matrices and on stacks of per-mode
    blocks (leading axes)."""
    if len(Ks) != 4 or len(s_pts) != 4:
        raise ValueError("four interpolation points")
    n = Ks[0].shape[-1]
    I = np.broadcast_to(np.eye(n, dtype=np.complex128), Ks[0].shape)
    cols = [np.concatenate([s * K, K, s * I, I], axis=-2) for K, s in zip(Ks, s_pts)]
    M = np.concatenate(cols, axis=-1)                                  # (..., 4n, 4n)
    rhs = np.concatenate([s * s * K for K, s in zip(Ks, s_pts)], axis=-1)  # (..., n, 4n)
    X = np.swapaxes(np.linalg.solve(np.swapaxes(M, -1, -2), np.swapaxes(rhs, -1, -2)), -1, -2)
    return tuple(X[..., :, k * n:(k + 1) * n] for k in range(4))


def r22(B1, B0, A1, A0, s):
    """The second-order rational function at s (dense)."""
    n = B1.shape[-1]
    return np.linalg.solve(s * s * np.eye(n) - s * B1 - B0, s * A1 + A0)


# Relative singular-value level below which directions of the DtN maps are
# left out of the second-order interpolation (see box_second).
SECOND_ORDER_TAU = 1e-2


def dominant_subspace(Ks, tau=SECOND_ORDER_TAU) -> np.ndarray:
    """Real orthonormal basis U (n x r) of the directions in which the maps
    K(s_j) act above tau times their largest singular value: the eigenvectors
    of Re sum_j K_j K_j^H (= sum_j Re K_j Re K_j^T + Im K_j Im K_j^T) whose
    eigenvalues exceed tau^2 times the largest.  The span holds the real and
    imaginary parts of the columns, so it is closed under conjugation."""
    G = sum((K @ K.conj().T).real for K in Ks)
    w, V = np.linalg.eigh(G)
    return V[:, w > tau * tau * w.max()]


def box_second(shape, h, R, s_pts, L=None, tau=SECOND_ORDER_TAU) -> BoxOperators:
    """Second-order coefficients of the dense box form by four-point
    interpolation of the DtN map (Sec. 3.3; the paper gives no stability
    theorem for this order and does not say how the coefficients are formed).

    For R >= 2 the maps are numerically rank-deficient: the deeper boundary
    layers reach the exterior only through the small outer stencil weights,
    and the singular values fall into two groups with a wide gap between
    them (the boundary's outermost layer above about 0.09 of the largest,
    the rest below about 1e-3, for R = 2 and 3, h = 0.1 to 0.3).  The 4n
    system is then singular to working precision.  The
    interpolation runs in the dominant subspace U of the four maps: the
    reduced maps U^T K_j U are interpolated, and each coefficient is lifted
    as U X U^T.  The auxiliary variables then live in span(U): they start at
    zero and every source and coupling maps into it, so the dropped
    directions stay inert.  When no direction falls below tau (R = 1) this is
    the plain 4n solve."""
    gamma = gamma_points(shape, R)
    Ks = [dtn_box(shape, h, R, s, L) for s in s_pts]
    U = dominant_subspace(Ks, tau)
    if U.shape[1] == len(gamma):
        B1, B0, A1, A0 = interp_second(Ks, s_pts)
    else:
        red = interp_second([U.T @ K @ U for K in Ks], s_pts)
        B1, B0, A1, A0 = (U @ X @ U.T for X in red)
    return BoxOperators("second", gamma, B1=B1, B0=B0, A1=A1, A0=A0, C=B1 @ A1 + A0)


# ---------------------------------------------------------------------------
# Face form
# ---------------------------------------------------------------------------

# face f = 2*axis + side; axis 0 = x, 1 = y, 2 = z; side 0 = low, 1 = high.
# array axes of psi[z, y, x]: x -> 2, y -> 1, z -> 0.
FACE_ARRAY_AXIS = {0: 2, 1: 1, 2: 0}


def face_geometry(shape, f: int):
    """(array axis normal to face f, side, transverse array axes in array order)."""
    axis = FACE_ARRAY_AXIS[f // 2]
    side = f % 2
    trans = tuple(a for a in range(3) if a != axis)
    return axis, side, trans


def face_extract(psi: np.ndarray, f: int, R: int) -> np.ndarray:
    """E_f psi: the R x n1 x n2 slab of face f (layer 0 outermost)."""
    axis, side, trans = face_geometry(psi.shape[:3], f)
    n = psi.shape[axis]
    idx = [l if side == 0 else n - 1 - l for l in range(R)]
    slab = np.take(psi, idx, axis=axis)           # layer axis sits at ``axis``
    return np.moveaxis(slab, axis, 0)


def face_scatter_add(out: np.ndarray, slab: np.ndarray, f: int, R: int) -> None:
    """out += E_f^T slab."""
    axis, side, trans = face_geometry(out.shape[:3], f)
    n = out.shape[axis]
    for l in range(R):
        i = l if side == 0 else n - 1 - l
        sl = [slice(None)] * out.ndim
        sl[axis] = i
        out[tuple(sl)] += slab[l]


def symbol_grid(P: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(P) / P


def default_symbol_points(s: float, h: float, w_max: int) -> int:
    need = max(64, 4 * (w_max + 1), int(math.ceil(60.0 / (math.sqrt(s) * h))))
    P = 64
    while P < need:
        P *= 2
    return P


def face_kernel_from_symbol(sym: np.ndarray, w: int) -> np.ndarray:
    """Fourier coefficients k(p), |p|_inf <= w, of a (P, P, R, R) symbol on the
    uniform theta grid (trapezoidal rule = inverse 2D DFT); returned as
    (R, R, 2w+1, 2w+1) with offset index p + w."""
    P = sym.shape[0]
    R = sym.shape[2]
    coef = np.fft.ifft2(sym, axes=(0, 1))          # coef[p mod P]
    out = np.empty((R, R, 2 * w + 1, 2 * w + 1), dtype=np.complex128)
    for a in range(2 * w + 1):
        for b in range(2 * w + 1):
            out[:, :, a, b] = coef[(a - w) % P, (b - w) % P]
    return out


def fejer_window(w: int) -> np.ndarray:
    t = 1.0 - np.abs(np.arange(-w, w + 1)) / (w + 1.0)
    return np.outer(t, t)


@dataclasses.dataclass
class FaceOperators:
    """Per-face operators shared by all six faces (uniform spacing).

    ``kernel``: (R, R, 2w+1, 2w+1) transverse kernel of M (zeroth) or B
    (first) in layer-by-layer blocks.  ``a``: (R, R) normal-line block of A
    (first order).  ``q``: (R, R) Lyapunov weight (H_gs H_gs^T)^{-1}.
    """
    order: str
    R: int
    w: int
    kernel: np.ndarray
    a: Optional[np.ndarray] = None
    q: Optional[np.ndarray] = None
    symbol: Optional[np.ndarray] = None
    # second order: kernels of B1, B0, A1 and C = B1 A1 + A0 (per-mode products)
    kernels2: Optional[dict] = None


def face_symbol_k(s: float, h: float, R: int, P: int) -> np.ndarray:
    th = symbol_grid(P)
    tau = greens.transverse_shift(th[:, None], th[None, :], h, R)
    return greens.halfline_symbol(tau - 1j * s, h, R)


def face_zeroth(h, R, s0, w, P=None, window=True) -> FaceOperators:
    if P is None:
        P = default_symbol_points(s0, h, w)
    sym = face_symbol_k(s0, h, R, P)
    ker = face_kernel_from_symbol(sym, w)
    if window:
        ker = ker * fejer_window(w)[None, None]
    return FaceOperators("zeroth", R, w, ker, symbol=sym)


def face_first(h, R, s1, w, P=None, window=True) -> FaceOperators:
    """b^(theta) = s1 I - a k^(theta; s1)^{-1}, a = -i H_gs H_gs^T (per mode
    version of the first-order stability theorem)."""
    if P is None:
        P = default_symbol_points(s1, h, w)
    Hgs = greens.coupling_1d(h, R)
    HH = Hgs @ Hgs.T
    a = -1j * HH
    k1 = face_symbol_k(s1, h, R, P)
    # a k^{-1} = (k^{-T} a^T)^T ; per mode
    akinv = np.transpose(np.linalg.solve(np.transpose(k1, (0, 1, 3, 2)), np.broadcast_to(a.T, k1.shape)), (0, 1, 3, 2))
    bsym = s1 * np.eye(R)[None, None] - akinv
    ker = face_kernel_from_symbol(bsym, w)
    if window:
        ker = ker * fejer_window(w)[None, None]
    return FaceOperators("first", R, w, ker, a=a, q=np.linalg.inv(HH), symbol=bsym)


def face_second(h, R, s_pts, w, P=None, window=True) -> FaceOperators:
    """Second-order face operators: the four-point interpolation of Sec. 3.3
    applied mode by mode to the half-line symbol k^(theta; s), giving symbols
    b1, b0, a1, a0 and c = b1 a1 + a0, whose windowed sections are the
    kernels."""
    if P is None:
        P = max(default_symbol_points(s, h, w) for s in s_pts)
    Ks = [face_symbol_k(s, h, R, P) for s in s_pts]
    b1, b0, a1, a0 = interp_second(Ks, s_pts)
    syms = {"b1": b1, "b0": b0, "a1": a1, "c": b1 @ a1 + a0}
    kers = {}
    for name, sym in syms.items():
        ker = face_kernel_from_symbol(sym, w)
        if window:
            ker = ker * fejer_window(w)[None, None]
        kers[name] = ker
    return FaceOperators("second", R, w, kers["b1"], kernels2=kers, symbol=syms)


def face_apply_kernel(ker: np.ndarray, slab: np.ndarray) -> np.ndarray:
    """Toeplitz section: out[l, i] = sum_{l', j} k_{l,l'}(i - j) slab[l', j] over
    the slab, written as a sum over offsets p = j - i of k(-p) slab[i + p]
    (plain loops over offsets; the kernels here are even, k(p) = k(-p))."""
    R = ker.shape[0]
    w = (ker.shape[2] - 1) // 2
    n1, n2 = slab.shape[1], slab.shape[2]
    out = np.zeros_like(slab)
    extra = slab.shape[3:]
    for l in range(R):
        for lp in range(R):
            for a in range(-w, w + 1):
                if abs(a) >= n1:
                    continue
                for b in range(-w, w + 1):
                    if abs(b) >= n2:
                        continue
                    kv = ker[l, lp, -a + w, -b + w]
                    if kv == 0:
                        continue
                    # out[i, j] += kv * slab[i + a, j + b]
                    i0, i1 = max(0, -a), min(n1, n1 - a)
                    j0, j1 = max(0, -b), min(n2, n2 - b)
                    out[l, i0:i1, j0:j1] += kv * slab[lp, i0 + a:i1 + a, j0 + b:j1 + b]
    return out


def face_apply_local(mat: np.ndarray, slab: np.ndarray) -> np.ndarray:
    """out[l] = sum_{l'} mat[l, l'] slab[l'] (normal-line block, identity along the face)."""
    return np.tensordot(mat, slab, axes=([1], [0]))


def face_dense_section(ops: FaceOperators, n1: int, n2: int) -> np.ndarray:
    """Dense (R n1 n2)^2 matrix of the section (small faces only; for tests)."""
    R = ops.R
    m = R * n1 * n2
    D = np.zeros((m, m), dtype=np.complex128)
    e = np.zeros((R, n1, n2), dtype=np.complex128)
    for j in range(m):
        e[:] = 0
        e.reshape(-1)[j] = 1
        D[:, j] = face_apply_kernel(ops.kernel, e).reshape(-1)
    return D
