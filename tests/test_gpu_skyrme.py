"""Mean field with the long-range TDHF terms (Sec. 4.3): Yukawa and Coulomb
fields of the density solved on the device by conjugate gradients, against
the oracle's exact sparse solves.

Tolerance: the solves stop at relative residual tol = 1e-14, so the fields
carry a relative error of at most cond(A) * tol, with cond(A) below 1e3 on
these boxes (the ratio of the extreme eigenvalues of -Delta_h + mu^2).  The
potential is checked at 1e-11 of its largest value; the stepped states,
which see the potential through dt-weighted products, at the FP64 bar.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import integrate, poisson
from paper_1908_02456_amd import workloads as W

pytestmark = pytest.mark.gpu

MF = dict(t0=-1.0, t3=0.5, v0=-0.8, a=0.7, e2=0.3, tol=1e-14, maxit=3000)


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02456_amd.solver import Solver
    return Solver


def _setup(shape, h, dt, R, order, **kw):
    return integrate.make_setup(shape, h, dt, R, order, t0=MF["t0"], t3=MF["t3"], v0=MF["v0"], a_y=MF["a"],
                                e2=MF["e2"], **kw)


@pytest.mark.parametrize("shape,R,batch", [((11, 12, 10), 1, 3), ((10, 9, 12), 2, 2), ((13, 11, 11), 3, 1)])
def test_effective_potential_matches_oracle(shape, R, batch):
    print("case: skyrme veff", shape, R, batch, flush=True)
    Solver = _gpu()
    h = 0.3
    s = Solver(shape, h, 0.002, radius=R, order="dirichlet", batch=batch, meanfield=MF)
    full = shape + (batch,) if batch > 1 else shape
    psi0 = W.random_complex(full, seed=4)
    V = W.random_potential(shape, seed=5)
    st = _setup(shape, h, 0.002, R, "dirichlet")
    ref = V + integrate.meanfield(st, psi0)
    got = s.effective_potential(torch.from_numpy(psi0).cuda(), torch.from_numpy(V).cuda()).cpu().numpy()
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()
    n_eval, iy, ic = s.potential_iterations()
    assert n_eval == 1 and iy >= 1 and ic >= 1
    if R == 1:
        # the sine-transform preconditioner is the exact inverse for R = 1
        assert iy <= 3 and ic <= 3, (iy, ic)
    # the same state again: the solves start from their own solution
    s.effective_potential(torch.from_numpy(psi0).cuda(), torch.from_numpy(V).cuda())
    n2, iy2, ic2 = s.potential_iterations()
    print("  iterations: first %d + %d, again %d + %d" % (iy, ic, iy2 - iy, ic2 - ic), flush=True)
    assert n2 == 2 and iy2 - iy <= 3 and ic2 - ic <= 3


def test_effective_potential_fp32_state():
    Solver = _gpu()
    shape, h = (10, 11, 12), 0.3
    s = Solver(shape, h, 0.002, order="dirichlet", batch=2, meanfield=MF, dtype="c64")
    psi0 = W.random_complex(shape + (2,), seed=6)
    V = W.random_potential(shape, seed=7)
    ref = V + integrate.meanfield(_setup(shape, h, 0.002, 1, "dirichlet"), psi0)
    got = s.effective_potential(torch.from_numpy(psi0).to(torch.complex64).cuda(),
                                torch.from_numpy(V).float().cuda()).cpu().numpy()
    # the density comes from the complex64 state; the solves are FP64
    assert np.abs(got - ref).max() < 1e-5 * np.abs(ref).max()


def test_zero_density_gives_the_bare_potential():
    Solver = _gpu()
    shape = (9, 10, 11)
    s = Solver(shape, 0.3, 0.002, order="dirichlet", meanfield=MF)
    V = torch.from_numpy(W.random_potential(shape, seed=8)).cuda()
    s.effective_potential(torch.from_numpy(W.random_complex(shape, seed=9)).cuda(), V)
    got = s.effective_potential(torch.zeros(shape, dtype=torch.complex128, device="cuda"), V)
    assert torch.equal(got, V)  # the warm start is dropped and W = 0 exactly


@pytest.mark.parametrize("path,order,window,batch,steps", [("staged", "first", 1, 3, 4), ("auto", "first", 0, 4, 5),
                                                            ("auto", "zeroth", 0, 2, 4)])
def test_stepping_with_long_range_mean_field_matches_oracle(path, order, window, batch, steps):
    print("case: skyrme step", path, order, window, batch, steps, flush=True)
    Solver = _gpu()
    shape, h, dt = (12, 11, 13), 0.3, 0.004
    st = _setup(shape, h, dt, 1, order, s0=1.5, s1=1.5, window=window)
    psi0 = W.random_complex(shape + (batch,), seed=10) * 0.5
    V = W.random_potential(shape, seed=11)
    ref_psi, ref_aux, _ = integrate.run(st, psi0, V, steps)
    s = Solver(shape, h, dt, order=order, s0=1.5, s1=1.5, window=window, batch=batch, meanfield=MF, path=path)
    if path == "auto":
        assert s.use_fused  # the fused orbital-batch path
    psi = torch.from_numpy(psi0).cuda().contiguous()
    aux = s.new_aux()
    s.step(psi, aux, torch.from_numpy(V).cuda(), steps)
    err = np.abs(psi.cpu().numpy() - ref_psi).max() / np.abs(ref_psi).max()
    print("  err %.2e" % err, flush=True)
    assert err < 1e-12, err
    if order == "first":
        ref_flat = integrate.pack_aux(st, ref_aux)
        got = aux.cpu().numpy()[:ref_flat.size]
        assert np.abs(got - ref_flat).max() < 1e-12 * np.abs(ref_flat).max()


def test_full_size_potentials_satisfy_the_discrete_equations():
    # the TDHF batch at full size (32 oscillator orbitals, 96^3): the device's
    # Yukawa and Coulomb fields, from two contexts with one term each, solve
    # the oracle's sparse Helmholtz and Poisson systems built from the same
    # state's density.  The solves stop at a relative residual of 1e-12; the
    # true residual is checked at 1e-10.
    Solver = _gpu()
    n, nb, h = 96, 32, 0.2
    print("case: skyrme 96^3 x 32 residuals", flush=True)
    orb = W.oscillator_orbitals((n,) * 3, h, nb, seed=3)
    psi = torch.from_numpy(orb).cuda().contiguous()
    rho = (np.abs(orb) ** 2).sum(axis=3)
    base = dict(t0=0.0, t3=0.0, tol=1e-12, maxit=200)
    A = poisson.neg_laplacian((n,) * 3, h, 1)
    for name, extra, mu2, scale in (("yukawa", dict(v0=-0.5, a=0.7), 1 / 0.7 ** 2, 4 * np.pi * -0.5 * 0.7),
                                    ("coulomb", dict(e2=0.1), 0.0, 2 * np.pi * 0.1)):
        s = Solver((n,) * 3, h, 0.002, order="first", window=0, batch=nb, meanfield=dict(base, **extra))
        Wd = s.effective_potential(psi).cpu().numpy().ravel()
        print("  %s iterations" % name, s.potential_iterations(), flush=True)
        b = scale * rho.ravel()
        res = A @ Wd + mu2 * Wd - b
        rel = np.linalg.norm(res) / np.linalg.norm(b)
        print("  %s relative residual %.2e" % (name, rel), flush=True)
        assert rel < 1e-10, (name, rel)
        del s
        torch.cuda.empty_cache()
