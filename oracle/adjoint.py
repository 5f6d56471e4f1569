"""Discrete adjoint of the Taylor-4 stepping map.

Test infrastructure: part of the FP64 oracle, not of the product path.

The step of Sec. 4 applied to the linear dynamics of Sec. 3 is the matrix
polynomial P(dt L) = sum_{k<=4} (dt L)^k / k! of the generator L.  For a real
objective J of the final state, write its gradient with respect to a complex
vector z as g = dJ/dRe z + i dJ/dIm z, so that dJ = Re <g, dz>.  Then:

* states: lambda_n = P(dt L)^H lambda_{n+1} = P(dt L^H) lambda_{n+1}, since P
  has real coefficients;
* potential: L depends on V only through the psi block, where dL y = -i dV y.
  Differentiating the polynomial term by term,
    dP(X) = sum_k (1/k!) sum_{j<k} X^j dX X^(k-1-j),
  so with a_j = (L^H)^j lambda_{n+1} and b_m = L^m z_n,
    dJ/dV_p += sum_k dt^k/k! sum_{j<k} Im(conj(a_j[p]) b_{k-1-j}[p])
  over the psi components.

L^H is formed block by block from the definition of L (first order:
L = [[-iH, -iE^T], [A E, B]], so L^H = [[iH, E^T A^H], [iE, B^H]]; zeroth order:
L = -i(H + E^T M E), so L^H = i(H + E^T M^H E)).  Nothing here reuses the
forward map in a rescaled form.

Objectives: the probability left in the box, J = h^3 sum |psi_N|^2, and the
energy J = h^3 Re <psi_N, H psi_N> (H the box Hamiltonian with the potential,
no boundary term), for which dJ/dV also has the explicit part h^3 |psi_N|^2.
"""
from __future__ import annotations

import math

import numpy as np

from . import dtn
from .integrate import (Setup, _axpy_aux, _copy_aux, _scale_aux, _gather_gamma, _scatter_gamma,
                        generator, taylor4_step, zero_aux)
from .stencil import apply_H


def _adjoint_kernel(ker: np.ndarray) -> np.ndarray:
    """Kernel of the adjoint Toeplitz section: B[(l,i),(l',j)] = k_{l,l'}(i-j)
    gives B^H[(l,i),(l',j)] = conj(k_{l',l}(j-i))."""
    return np.conj(ker.transpose(1, 0, 2, 3)[:, :, ::-1, ::-1])


def generator_adjoint(st: Setup, lam: np.ndarray, mu, V: np.ndarray):
    """L^H applied to (lam, mu); returns (d_lam, d_mu)."""
    if st.t0 is not None:
        raise NotImplementedError("the mean field makes the step nonlinear")
    periodic = st.order == "periodic"
    dl = 1j * apply_H(lam, V, st.h, st.R, periodic=periodic)
    dm = None
    if st.order == "zeroth":
        if st.form == "box":
            src = st.box.M.conj().T @ _gather_gamma(st, lam)
            _scatter_gamma(st, dl, 1j * src)
        else:
            kh = _adjoint_kernel(st.faces.kernel)
            for f in range(6):
                slab = dtn.face_extract(lam, f, st.R)
                dtn.face_scatter_add(dl, 1j * dtn.face_apply_kernel(kh, slab), f, st.R)
    elif st.order == "first":
        if st.form == "box":
            _scatter_gamma(st, dl, st.box.A.conj().T @ mu)
            dm = 1j * _gather_gamma(st, lam) + st.box.B.conj().T @ mu
        else:
            kh = _adjoint_kernel(st.faces.kernel)
            ah = st.faces.a.conj().T
            dm = []
            for f in range(6):
                dtn.face_scatter_add(dl, dtn.face_apply_local(ah, mu[f]), f, st.R)
                slab = dtn.face_extract(lam, f, st.R)
                dm.append(1j * slab + dtn.face_apply_kernel(kh, mu[f]))
    return dl, dm


def inner(u, g, v, f) -> complex:
    """<(u, g), (v, f)> = sum conj(u) v + sum conj(g) f."""
    s = np.vdot(u, v)
    if g is not None:
        if isinstance(g, list):
            s += sum(np.vdot(a, b) for a, b in zip(g, f))
        else:
            s += np.vdot(g, f)
    return s


def objective(st: Setup, psi: np.ndarray, V: np.ndarray, kind: str):
    """(J, dJ/dpsi, explicit dJ/dV) for kind 'prob' or 'energy'."""
    h3 = st.h ** 3
    if kind == "prob":
        return h3 * float(np.sum(np.abs(psi) ** 2)), 2.0 * h3 * psi, np.zeros(V.shape)
    if kind == "energy":
        Hpsi = apply_H(psi, V, st.h, st.R, periodic=st.order == "periodic")
        J = h3 * float(np.real(np.vdot(psi, Hpsi)))
        return J, 2.0 * h3 * Hpsi, h3 * np.abs(psi) ** 2
    raise ValueError(kind)


def adjoint_run(st: Setup, psi0: np.ndarray, V: np.ndarray, steps: int, kind: str = "prob"):
    """J after ``steps`` steps from (psi0, f = 0), and its gradients with respect
    to psi0 (complex, convention above) and to V (real, per point)."""
    if psi0.ndim != 3:
        raise NotImplementedError("one orbital")
    states = [(psi0.astype(np.complex128), zero_aux(st))]
    for _ in range(steps):
        states.append(taylor4_step(st, *states[-1], V))
    J, lam, gV = objective(st, states[-1][0], V, kind)
    mu = zero_aux(st)
    dt = st.dt
    for n in range(steps - 1, -1, -1):
        z, fz = states[n]
        b = [(z, fz)]
        for _ in range(3):
            b.append(generator(st, *b[-1], V))
        a = [(lam, mu)]
        for _ in range(4):
            a.append(generator_adjoint(st, *a[-1], V))
        for k in range(1, 5):
            ck = dt ** k / math.factorial(k)
            for j in range(k):
                gV = gV + ck * np.imag(np.conj(a[j][0]) * b[k - 1 - j][0])
        new_lam, new_mu = lam.copy(), _copy_aux(mu)
        for k in range(1, 5):
            ck = dt ** k / math.factorial(k)
            new_lam = new_lam + ck * a[k][0]
            new_mu = _axpy_aux(ck, a[k][1], new_mu)
        lam, mu = new_lam, new_mu
    return J, lam, gV


def objective_value(st: Setup, psi0: np.ndarray, V: np.ndarray, steps: int, kind: str = "prob") -> float:
    """J alone (forward run), for finite differences."""
    psi, aux = psi0.astype(np.complex128), zero_aux(st)
    for _ in range(steps):
        psi, aux = taylor4_step(st, psi, aux, V)
    return objective(st, psi, V, kind)[0]
