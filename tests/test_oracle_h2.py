"""Pins of the oracle's H2 objective for the first-order interpolation point
(Sec. 5 proposal, face form, R = 1).  No GPU."""
import math

import numpy as np
import pytest
from scipy import integrate as sint

from oracle import dtn, greens, h2


def test_axis_symbol_is_the_limit_from_the_right_half_plane():
    # k^(theta; delta + i omega) -> k^_axis as delta -> 0+, linearly in delta,
    # on and off the cut of the exterior spectrum
    h = 0.2
    tau = np.array([0.0, 7.0, 31.0, 77.0])[:, None]
    omega = np.array([-140.0, -60.0, -31.5, -20.0, -3.0, 0.5, 40.0])[None, :]
    ka = h2.halfline_symbol_axis(tau, omega, h)
    errs = []
    for d in (1e-4, 1e-5, 1e-6):
        kg = greens.halfline_symbol(tau - 1j * (d + 1j * omega), h, 1)[..., 0, 0]
        errs.append(np.abs(kg - ka).max() / np.abs(ka).max())
    assert errs[2] < 1e-6
    assert 5 < errs[0] / errs[1] < 20 and 5 < errs[1] / errs[2] < 20  # first order in delta


def test_axis_symbol_off_the_cut_equals_the_general_symbol():
    # b = 1 + h^2 (tau + omega) outside [-1, 1]: real roots, no branch choice
    h = 0.25
    tau = np.array([3.0, 12.0])[:, None]
    omega = np.array([-100.0, -60.0, 5.0, 80.0])[None, :]
    b = 1 + h * h * (tau + omega)
    assert np.all(np.abs(b) > 1)
    ka = h2.halfline_symbol_axis(tau, omega, h)
    kg = greens.halfline_symbol((tau + omega).astype(complex), h, 1)[..., 0, 0]
    assert np.abs(ka - kg).max() < 1e-13 * np.abs(kg).max()


@pytest.mark.parametrize("a,b", [(-156.25j, -3.0 + 2.0j), (2.0, -0.5 - 10.0j), (1 + 1j, -40.0 + 75.0j)])
def test_frequency_rule_on_a_one_pole_closed_form(a, b):
    omega, weight = h2.frequency_nodes(0.2, 4096)
    q = np.sum(np.abs(a / (1j * omega - b)) ** 2 * weight) / (2 * math.pi)
    assert abs(q - h2.one_pole_h2(a, b)) < 1e-12 * h2.one_pole_h2(a, b)


def test_kernel_symbol_inverts_the_kernel_construction():
    # a trigonometric polynomial of degree <= w survives kernel -> symbol exactly
    P, w = 16, 3
    th = dtn.symbol_grid(P)
    rng = np.random.default_rng(1)
    c = rng.standard_normal((2 * w + 1, 2 * w + 1)) + 1j * rng.standard_normal((2 * w + 1, 2 * w + 1))
    p = np.arange(-w, w + 1)
    e = np.exp(-1j * np.outer(th, p))
    sym = e @ c @ e.T
    ker = dtn.face_kernel_from_symbol(sym[:, :, None, None], w)
    assert np.abs(ker[0, 0] - c).max() < 1e-13 * np.abs(c).max()
    assert np.abs(h2.kernel_symbol(ker, P) - sym).max() < 1e-13 * np.abs(sym).max()


def test_objective_matches_adaptive_quadrature_per_mode():
    # one mode's integral by adaptive quadrature split at the branch points,
    # against the tan-mapped midpoint rule at growing N
    h, s1, w = 0.2, 3.0, 1
    fo = dtn.face_first(h, 1, s1, w)
    a = fo.a[0, 0]
    P = 8
    bw = h2.kernel_symbol(fo.kernel, P)
    th = dtn.symbol_grid(P)
    i, j = 1, 3
    tau = float(greens.transverse_shift(th[i], th[j], h, 1))
    f = lambda om: abs(h2.halfline_symbol_axis(tau, om, h) - a / (1j * om - bw[i, j])) ** 2
    br = sorted([-tau, -tau - 2.0 / (h * h)])
    pieces = [(-np.inf, br[0]), (br[0], br[1]), (br[1], np.inf)]
    ref = sum(sint.quad(f, lo, hi, limit=400, epsabs=0, epsrel=1e-11)[0] for lo, hi in pieces) / (2 * math.pi)
    errs = []
    for N in (1024, 8192, 65536):
        omega, weight = h2.frequency_nodes(h, N)
        val = np.sum(f(omega) * weight) / (2 * math.pi)
        errs.append(abs(val - ref) / ref)
    assert errs[-1] < 1e-5 and errs[-1] < errs[0], errs


def test_objective_has_an_interior_minimum():
    # J(s1) falls from small s1, rises again for large s1 (b_w -> the
    # two-term expansion at infinity): the minimiser is finite
    h = 0.2
    js = [h2.h2_objective(h, s, 0, P=16, N=512) for s in (1.0, 100.0, 10000.0)]
    assert js[1] < js[0] and js[1] < js[2]
    assert all(v > 0 for v in js)
