"""Pins of the oracle's long-range TDHF potentials (Sec. 4.3: Yukawa and
Coulomb fields from the Helmholtz and Poisson problems).  No GPU."""
import math

import numpy as np
import pytest

from oracle import poisson
from oracle.stencil import dense_H


@pytest.mark.parametrize("R", [1, 2, 3])
def test_operator_is_twice_the_kinetic_block(R):
    # -Delta_h against the kinetic part of the oracle's box Hamiltonian,
    # built by an independent routine: H(V = 0) = -(1/2) Delta_h
    shape, h = (7, 8, 9), 0.3
    A = poisson.neg_laplacian(shape, h, R).toarray()
    H = dense_H(shape, np.zeros(shape), h, R)
    assert np.abs(A - 2 * H).max() < 1e-12 * np.abs(A).max()


def test_sine_modes_are_solved_exactly():
    # R = 1, zero outside: sin(k pi (j + 1) / (n + 1)) per axis is an
    # eigenvector of -Delta_h with eigenvalue sum (2 / h^2)(1 - cos(k pi / (n + 1)))
    shape, h = (7, 9, 8), 0.25
    ks = (2, 3, 1)
    axes = [np.sin(k * math.pi * (np.arange(n) + 1) / (n + 1)) for k, n in zip(ks, shape)]
    f = axes[0][:, None, None] * axes[1][None, :, None] * axes[2][None, None, :]
    lam = sum(2.0 / h ** 2 * (1 - math.cos(k * math.pi / (n + 1))) for k, n in zip(ks, shape))
    e2 = 1.7
    Wc = poisson.coulomb(f, h, 1, e2)
    assert np.abs(Wc - 2 * math.pi * e2 * f / lam).max() < 1e-13 * np.abs(Wc).max()
    v0, a = 0.8, 0.6
    Wy = poisson.yukawa(f, h, 1, v0, a)
    ref = 4 * math.pi * v0 * a * f / (lam + 1 / a ** 2)
    assert np.abs(Wy - ref).max() < 1e-13 * np.abs(ref).max()


def test_coulomb_is_the_long_range_limit_of_yukawa():
    # V0 a = e^2 / 2 and a -> infinity turns the Helmholtz problem into the
    # Poisson problem: the difference falls like 1/a^2
    shape, h, e2 = (8, 9, 7), 0.3, 1.3
    rng = np.random.default_rng(2)
    rho = rng.uniform(0, 1, shape)
    Wc = poisson.coulomb(rho, h, 2, e2)
    errs = []
    for a in (10.0, 100.0):
        Wy = poisson.yukawa(rho, h, 2, e2 / (2 * a), a)
        errs.append(np.abs(Wy - Wc).max() / np.abs(Wc).max())
    assert errs[1] < 1e-3 and 50 < errs[0] / errs[1] < 200, errs


def test_yukawa_closed_form_against_radial_quadrature():
    from scipy import integrate as si
    q, sig, v0, a = 2.0, 0.5, 1.3, 0.4
    k = 1 / a
    rho = lambda r: q * (2 * math.pi * sig * sig) ** -1.5 * math.exp(-r * r / (2 * sig * sig))
    for r in (0.1, 0.7, 1.5):
        f = lambda rp: rp * rho(rp) * (math.exp(-k * abs(r - rp)) - math.exp(-k * (r + rp)))
        val = si.quad(f, 0, 20, points=[r], limit=200, epsabs=0, epsrel=1e-12)[0]
        ref = v0 * a * 2 * math.pi / (k * r) * val
        assert abs(poisson.yukawa_gaussian(r, q, sig, v0, a) / ref - 1) < 1e-12


@pytest.mark.slow
def test_yukawa_field_of_a_gaussian_converges_to_the_continuum():
    # discrete field of a Gaussian density (R = 1) against the continuum
    # screened potential, inside a box 4 ranges beyond the compared region;
    # the error falls with h at close to second order (3.4x per halving here)
    R, ratio = 1, 3.0
    q, sig, v0, a = 2.0, 0.5, 1.3, 0.4
    errs = []
    for n, h in ((17, 0.4), (33, 0.2)):
        x = (np.arange(n) - (n - 1) / 2) * h
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        rr = np.sqrt(X * X + Y * Y + Z * Z)
        rho = q * (2 * math.pi * sig * sig) ** -1.5 * np.exp(-rr * rr / (2 * sig * sig))
        W = poisson.yukawa(rho, h, R, v0, a)
        m = (rr > 0.05) & (rr < 1.5)
        ref = poisson.yukawa_gaussian(rr[m], q, sig, v0, a)
        errs.append(np.abs(W[m] - ref).max() / np.abs(ref).max())
    assert errs[1] < 1e-2 and errs[0] / errs[1] > ratio, errs
