"""Pins of the oracle's discrete adjoint against the definition of the adjoint
and against central finite differences of the forward map (no GPU)."""
import math

import numpy as np
import pytest

from oracle import adjoint, integrate
from paper_1908_02456_amd import workloads as W


def _setups():
    return [
        ("dirichlet", dict(order="dirichlet")),
        ("periodic", dict(order="periodic")),
        ("zeroth-faces-w1", dict(order="zeroth", s0=1.5, window=1)),
        ("first-faces-w0", dict(order="first", s1=1.5, window=0)),
        ("first-faces-w2", dict(order="first", s1=1.0, window=2)),
        ("first-faces-R2", dict(order="first", s1=1.0, window=1, R=2)),
        ("zeroth-box", dict(order="zeroth", form="box", s0=1.0)),
        ("first-box", dict(order="first", form="box", s1=1.0)),
    ]


def _make(kw, shape):
    kw = dict(kw)
    R = kw.pop("R", 1)
    return integrate.make_setup(shape, 0.3, 0.01, R, **kw)


def _rand_aux(st, seed):
    aux = integrate.zero_aux(st)
    if aux is None:
        return None
    if isinstance(aux, list):
        return [W.random_complex(a.shape, seed=seed + i) - (0.5 + 0.5j) for i, a in enumerate(aux)]
    return W.random_complex(aux.shape, seed=seed) - (0.5 + 0.5j)


@pytest.mark.parametrize("name,kw", _setups())
def test_generator_adjoint_is_the_adjoint(name, kw):
    # <u, L v> = <L^H u, v> for random states (psi and aux parts)
    shape = (6, 7, 5) if "box" not in name else (6, 6, 6)
    st = _make(kw, shape)
    V = W.random_potential(shape, seed=3)
    u = W.random_complex(shape, seed=4) - (0.5 + 0.5j)
    v = W.random_complex(shape, seed=5) - (0.5 + 0.5j)
    gu, gv = _rand_aux(st, 10), _rand_aux(st, 20)
    Lv = integrate.generator(st, v, gv, V)
    LHu = adjoint.generator_adjoint(st, u, gu, V)
    lhs = adjoint.inner(u, gu, *Lv)
    rhs = adjoint.inner(*LHu, v, gv)
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0), (lhs, rhs)


@pytest.mark.parametrize("name,kw,kind", [
    ("first-faces-w1", dict(order="first", s1=1.5, window=1), "prob"),
    ("first-faces-w0", dict(order="first", s1=1.0, window=0), "energy"),
    ("zeroth-faces-w0", dict(order="zeroth", s0=2.0, window=0), "prob"),
    ("dirichlet", dict(order="dirichlet"), "energy"),
])
def test_adjoint_gradients_match_central_differences(name, kw, kind):
    shape = (5, 6, 7)
    st = _make(kw, shape)
    st.dt = 0.02
    steps = 6
    x = W.mesh(shape, st.h)
    V = -3.0 * np.exp(-(x[0] ** 2 + x[1] ** 2 + x[2] ** 2) / 2.0)
    psi0 = W.gaussian_packet(shape, st.h, center=(0.1, -0.2, 0.3), k=(1.0, 0.5, -0.7))
    J, gpsi, gV = adjoint.adjoint_run(st, psi0, V, steps, kind)
    assert abs(J - adjoint.objective_value(st, psi0, V, steps, kind)) < 1e-14 * abs(J)
    eps = 1e-5
    rng = np.random.default_rng(7)
    pts = [(0, 0, 0), (4, 5, 6), (2, 3, 3), (0, 3, 6)] + [tuple(rng.integers(0, s) for s in shape) for _ in range(4)]
    # central differences: truncation O(eps^2), rounding about 1e-16 |J| / eps
    floor = 100 * np.finfo(float).eps * abs(J) / eps
    scale_V = np.abs(gV).max()
    scale_p = np.abs(gpsi).max()
    for p in pts:
        dV = np.zeros(shape)
        dV[p] = eps
        fd = (adjoint.objective_value(st, psi0, V + dV, steps, kind)
              - adjoint.objective_value(st, psi0, V - dV, steps, kind)) / (2 * eps)
        assert abs(fd - gV[p]) < 1e-7 * scale_V + floor, ("V", p, fd, gV[p])
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            d = np.zeros(shape, dtype=np.complex128)
            d[p] = unit * eps
            fd = (adjoint.objective_value(st, psi0 + d, V, steps, kind)
                  - adjoint.objective_value(st, psi0 - d, V, steps, kind)) / (2 * eps)
            assert abs(fd - part(gpsi[p])) < 1e-7 * scale_p + floor, ("psi0", p, part.__name__, fd, gpsi[p])


def test_adjoint_periodic_free_closed_form():
    # periodic box, V = 0: the step is diagonal in Fourier space with factor
    # T(theta) = sum_k (-i dt sigma)^k / k!, so for J = h^3 sum |psi_N|^2 the
    # gradient is 2 h^3 F^-1 (|T|^(2N) F psi0)
    shape = (6, 8, 7)
    st = integrate.make_setup(shape, 0.4, 0.02, 1, "periodic")
    steps = 5
    psi0 = W.random_complex(shape, seed=9)
    V = np.zeros(shape)
    J, gpsi, gV = adjoint.adjoint_run(st, psi0, V, steps, "prob")
    th = [2 * np.pi * np.fft.fftfreq(n) for n in shape]
    TH = np.meshgrid(*th, indexing="ij")
    sigma = sum((1.0 - np.cos(t)) / st.h ** 2 for t in TH)
    y = -1j * st.dt * sigma
    T = 1 + y + y ** 2 / 2 + y ** 3 / 6 + y ** 4 / 24
    ref = 2 * st.h ** 3 * np.fft.ifftn(np.abs(T) ** (2 * steps) * np.fft.fftn(psi0))
    assert np.abs(gpsi - ref).max() < 1e-12 * np.abs(ref).max()
    Jref = st.h ** 3 * np.sum(np.abs(np.fft.ifftn(T ** steps * np.fft.fftn(psi0))) ** 2)
    assert abs(J - Jref) < 1e-12 * Jref
