"""Time stepping with the absorbing boundary conditions.

Test infrastructure: part of the FP64 oracle, not of the product path.

Dynamics (Sec. 3):
  zeroth order   d/dt psi = -i (H_{I,I} psi + E^T M E psi)
  first order    d/dt psi = -i H_{I,I} psi - i E^T f,   d/dt f = B f + A E psi
  plus two references without a condition: the box with zero values outside
  (Dirichlet, the I,I block alone) and the periodic box.
  In the face form E^T M E = sum_f E_f^T M_f E_f and the auxiliary variable is
  one slab per face, f = sum_f E_f^T f_f.

Integrator (Sec. 4, Taylor propagator): the paper truncates exp(-i dt H)
after the fourth power.  Its printed signs of the cubic and quartic terms are
garbled; the reading used is the Taylor polynomial itself,
  U = sum_{k=0..4} (dt L)^k / k!,
applied to the generator L of the (augmented) linear dynamics, evaluated as
z_0 = state, z_k = (dt / k) L z_{k-1}, new state = z_0 + ... + z_4.

Mean field (Sec. 4.3 with the simplified functional U = t0 rho + t3 rho^2,
rho = sum_j |phi_j|^2, optionally plus the Yukawa and Coulomb fields of rho
from :mod:`poisson`): rebuilt from the state at the start of each step and
held fixed across the four stages.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

from . import dtn, poisson
from .stencil import apply_H, laplacian


@dataclasses.dataclass
class Setup:
    shape: tuple                 # (nz, ny, nx)
    h: float
    dt: float
    R: int
    order: str                   # dirichlet | periodic | zeroth | first
    form: str = "faces"          # box | faces
    box: Optional[dtn.BoxOperators] = None
    faces: Optional[dtn.FaceOperators] = None
    t0: Optional[float] = None   # mean field U = t0 rho + t3 rho^2 when set
    t3: float = 0.0
    v0: float = 0.0              # Yukawa strength and range (with t0 set)
    a_y: float = 1.0
    e2: float = 0.0              # Coulomb e^2 (with t0 set)


def make_setup(shape, h, dt, R, order, form="faces", s0=1.0, s1=1.0, s2=math.inf,
               window=0, use_window=True, P=None, t0=None, t3=0.0, s_second=(1.0, 2.0, 3.0, 10.0),
               v0=0.0, a_y=1.0, e2=0.0) -> Setup:
    st = Setup(tuple(shape), h, dt, R, order, form, t0=t0, t3=t3, v0=v0, a_y=a_y, e2=e2)
    if order == "second":
        if form == "box":
            st.box = dtn.box_second(shape, h, R, s_second)
        else:
            st.faces = dtn.face_second(h, R, s_second, window, P=P, window=use_window)
        return st
    if order == "zeroth":
        if form == "box":
            st.box = dtn.box_zeroth(shape, h, R, s0)
        else:
            st.faces = dtn.face_zeroth(h, R, s0, window, P=P, window=use_window)
    elif order == "first":
        if form == "box":
            st.box = dtn.box_first(shape, h, R, s1, s2)
        else:
            if not math.isinf(s2):
                raise NotImplementedError("face form uses the theorem's (s1, inf) pair")
            st.faces = dtn.face_first(h, R, s1, window, P=P, window=use_window)
    return st


# ---------------------------------------------------------------------------
# Auxiliary variable containers
# ---------------------------------------------------------------------------

def face_shapes(shape, R):
    out = []
    for f in range(6):
        axis, side, trans = dtn.face_geometry(shape, f)
        out.append((R, shape[trans[0]], shape[trans[1]]))
    return out


def zero_aux(st: Setup, batch: Optional[int] = None):
    extra = () if batch is None else (batch,)
    if st.order == "second":
        one = Setup(st.shape, st.h, st.dt, st.R, "first", st.form, box=st.box, faces=st.faces)
        return (zero_aux(one, batch), zero_aux(one, batch))
    if st.order != "first":
        return None
    if st.form == "box":
        return np.zeros((len(st.box.gamma),) + extra, dtype=np.complex128)
    return [np.zeros(s + extra, dtype=np.complex128) for s in face_shapes(st.shape, st.R)]


def pack_aux(st: Setup, aux) -> np.ndarray:
    """Flat aux vector in the library's layout: box form [gamma][orb]; face form
    [face][layer][t_slow][t_fast][orb], faces in the order x-, x+, y-, y+, z-, z+."""
    if aux is None:
        return np.zeros(0, dtype=np.complex128)
    if isinstance(aux, tuple):  # second order: the f part, then the g part
        one = Setup(st.shape, st.h, st.dt, st.R, "first", st.form, box=st.box, faces=st.faces)
        return np.concatenate([pack_aux(one, aux[0]), pack_aux(one, aux[1])])
    if st.form == "box":
        return aux.reshape(-1)
    return np.concatenate([a.reshape(-1) for a in aux])


def unpack_aux(st: Setup, flat: np.ndarray, batch: Optional[int] = None):
    if st.order == "second":
        one = Setup(st.shape, st.h, st.dt, st.R, "first", st.form, box=st.box, faces=st.faces)
        half = flat.size // 2
        return (unpack_aux(one, flat[:half], batch), unpack_aux(one, flat[half:], batch))
    if st.order != "first":
        return None
    extra = () if batch is None else (batch,)
    if st.form == "box":
        return flat.reshape((len(st.box.gamma),) + extra).astype(np.complex128)
    out, off = [], 0
    for s in face_shapes(st.shape, st.R):
        n = int(np.prod(s + extra))
        out.append(flat[off:off + n].reshape(s + extra).astype(np.complex128))
        off += n
    return out


def _axpy_aux(a, x, y):
    """a * x + y for aux containers."""
    if x is None:
        return None
    if isinstance(x, tuple):
        return tuple(_axpy_aux(a, xi, yi) for xi, yi in zip(x, y))
    if isinstance(x, list):
        return [a * xi + yi for xi, yi in zip(x, y)]
    return a * x + y


def _scale_aux(a, x):
    if x is None:
        return None
    if isinstance(x, tuple):
        return tuple(_scale_aux(a, xi) for xi in x)
    if isinstance(x, list):
        return [a * xi for xi in x]
    return a * x


def _copy_aux(x):
    if x is None:
        return None
    if isinstance(x, tuple):
        return tuple(_copy_aux(xi) for xi in x)
    if isinstance(x, list):
        return [xi.copy() for xi in x]
    return x.copy()


# ---------------------------------------------------------------------------
# Generator and Taylor step
# ---------------------------------------------------------------------------

def meanfield(st: Setup, psi: np.ndarray) -> np.ndarray:
    """U = t0 rho + t3 rho^2 (+ W_Y + W_C) with rho = sum over orbitals of
    |phi_j|^2."""
    rho = np.abs(psi) ** 2
    if psi.ndim == 4:
        rho = rho.sum(axis=3)
    U = st.t0 * rho + st.t3 * rho * rho
    if st.v0 != 0.0:
        U = U + poisson.yukawa(rho, st.h, st.R, st.v0, st.a_y)
    if st.e2 != 0.0:
        U = U + poisson.coulomb(rho, st.h, st.R, st.e2)
    return U


def _gather_gamma(st, y):
    g = st.box.gamma
    return y[g[:, 0], g[:, 1], g[:, 2]]


def _scatter_gamma(st, out, vals):
    g = st.box.gamma
    out[g[:, 0], g[:, 1], g[:, 2]] += vals


def generator(st: Setup, y: np.ndarray, g, V: np.ndarray):
    """L(y, g) for the configured dynamics; returns (dy, dg)."""
    periodic = st.order == "periodic"
    dy = -1j * apply_H(y, V, st.h, st.R, periodic=periodic)
    dg = None
    if st.order == "zeroth":
        if st.form == "box":
            src = st.box.M @ _gather_gamma(st, y)
            _scatter_gamma(st, dy, -1j * src)
        else:
            for f in range(6):
                slab = dtn.face_extract(y, f, st.R)
                dtn.face_scatter_add(dy, -1j * dtn.face_apply_kernel(st.faces.kernel, slab), f, st.R)
    elif st.order == "first":
        if st.form == "box":
            _scatter_gamma(st, dy, -1j * g)
            dg = st.box.B @ g + st.box.A @ _gather_gamma(st, y)
        else:
            dg = []
            for f in range(6):
                dtn.face_scatter_add(dy, -1j * g[f], f, st.R)
                slab = dtn.face_extract(y, f, st.R)
                dg.append(dtn.face_apply_kernel(st.faces.kernel, g[f])
                          + dtn.face_apply_local(st.faces.a, slab))
    elif st.order == "second":
        # Sec. 3.3 dynamics written first-order in (psi, f, g) with
        # g = df/dt - A1 E psi (zero at t = 0 for zero exterior data):
        #   d psi/dt = -i H psi - i E^T f,  df/dt = g + A1 E psi,
        #   dg/dt = B1 g + B0 f + (B1 A1 + A0) E psi
        f, gg = g
        if st.form == "box":
            _scatter_gamma(st, dy, -1j * f)
            Ey = _gather_gamma(st, y)
            dg = (gg + st.box.A1 @ Ey, st.box.B1 @ gg + st.box.B0 @ f + st.box.C @ Ey)
        else:
            k = st.faces.kernels2
            dfs, dgs = [], []
            for fi in range(6):
                dtn.face_scatter_add(dy, -1j * f[fi], fi, st.R)
                slab = dtn.face_extract(y, fi, st.R)
                dfs.append(gg[fi] + dtn.face_apply_kernel(k["a1"], slab))
                dgs.append(dtn.face_apply_kernel(k["b1"], gg[fi]) + dtn.face_apply_kernel(k["b0"], f[fi])
                           + dtn.face_apply_kernel(k["c"], slab))
            dg = (dfs, dgs)
    return dy, dg


def taylor4_step(st: Setup, psi: np.ndarray, aux, V: np.ndarray):
    """One step of U = sum_{k<=4} (dt L)^k / k! on the state (psi, aux)."""
    Veff = V
    if st.t0 is not None:
        U = meanfield(st, psi)
        Veff = V + U
    y, g = psi, aux
    out_psi, out_aux = psi.copy(), _copy_aux(aux)
    for k in range(1, 5):
        dy, dg = generator(st, y, g, Veff)
        y = (st.dt / k) * dy
        g = _scale_aux(st.dt / k, dg)
        out_psi = out_psi + y
        out_aux = _axpy_aux(1.0, g, out_aux)
    return out_psi, out_aux


def run(st: Setup, psi0: np.ndarray, V: np.ndarray, steps: int, aux0=None,
        diag_every: int = 0):
    """Advance ``steps`` steps; returns (psi, aux, diagnostics list)."""
    psi = psi0.astype(np.complex128).copy()
    batch = psi.shape[3] if psi.ndim == 4 else None
    aux = aux0 if aux0 is not None else zero_aux(st, batch)
    diags = []
    if diag_every:
        diags.append(diagnostics(st, psi, aux, V))
    for n in range(steps):
        psi, aux = taylor4_step(st, psi, aux, V)
        if diag_every and (n + 1) % diag_every == 0:
            diags.append(diagnostics(st, psi, aux, V))
    return psi, aux, diags


# ---------------------------------------------------------------------------
# Diagnostics (Sec. 3 Lyapunov functionals; Sec. 4 norm and energy)
# ---------------------------------------------------------------------------

def norm(st: Setup, psi: np.ndarray) -> np.ndarray:
    """h^3 sum |psi|^2 (per orbital for a batch)."""
    a = np.abs(psi) ** 2
    return st.h ** 3 * a.sum(axis=(0, 1, 2))


def aux_energy(st: Setup, aux) -> np.ndarray:
    """f^* Q f (per orbital), Q = (H_{Gamma,II} H_{II,Gamma})^{-1}.  The
    second order has no Lyapunov functional in the paper: 0."""
    if aux is None or st.order == "second":
        return 0.0
    if st.form == "box":
        Qf = st.box.Q @ aux
        return np.real(np.sum(np.conj(aux) * Qf, axis=0))
    tot = 0.0
    for a in aux:
        Qa = dtn.face_apply_local(st.faces.q, a)
        tot = tot + np.real(np.sum(np.conj(a) * Qa, axis=(0, 1, 2)))
    return tot


def lyapunov(st: Setup, psi, aux) -> np.ndarray:
    """W = h^3 (psi^* psi + f^* Q f): the functional the stability theorems
    show to be non-increasing for the semi-discrete dynamics."""
    return norm(st, psi) + st.h ** 3 * aux_energy(st, aux)


def energy(st: Setup, psi: np.ndarray, V: np.ndarray) -> np.ndarray:
    """h^3 Re <psi, H_{I,I} psi> per orbital; with the mean field the
    interaction energy h^3 sum (t0 rho^2/2 + t3 rho^3/3) is added to the
    total (returned as the sum over orbitals plus that term)."""
    Hpsi = apply_H(psi, V, st.h, st.R, periodic=(st.order == "periodic"))
    e = st.h ** 3 * np.real(np.sum(np.conj(psi) * Hpsi, axis=(0, 1, 2)))
    if st.t0 is not None:
        rho = np.abs(psi) ** 2
        if psi.ndim == 4:
            rho = rho.sum(axis=3)
        e = np.sum(e) + st.h ** 3 * np.sum(st.t0 * rho ** 2 / 2 + st.t3 * rho ** 3 / 3)
    return e


def diagnostics(st, psi, aux, V):
    return {"norm": norm(st, psi), "lyapunov": lyapunov(st, psi, aux),
            "energy": energy(st, psi, V)}
