"""Graph capture of steps with the long-range mean field (Sec. 4.3): with a
fixed number of conjugate-gradient iterations per solve (pcg_fixed) a step
reads nothing on the host, so it can be captured in a HIP graph and
replayed.  Each case checks the fixed-iteration step against the adaptive
one, then replays a captured step several times, with eager work and
synchronisations between the replays, against eager steps of the same
states, and reads the device's iteration and convergence tallies.

Tolerance: the solves stop at relative residual 1e-14 and start from each
solver's own previous potential, so two solvers reach the same potential to
about cond * 1e-14 (cond below 1e3 here), and the states after a step,
which see the potential through dt, agree to 1e-12."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1908_02456_amd import workloads as W

pytestmark = pytest.mark.gpu

MF = dict(t0=-1.0, t3=0.5, v0=-0.8, a=0.7, e2=0.3, tol=1e-14, maxit=3000)
TOL = 1e-12

# (name, shape, R, batch, dtype, path, iterations per solve): the one-pass
# orbital sweep (complex64 orbitals), the two-stage orbital kernels
# (complex128 orbitals) and the staged path
CASES = [("onepass-orbitals", (18, 20, 22), 1, 3, "c64", "auto", 4),
         ("two-stage-orbitals", (14, 12, 16), 1, 2, "c128", "auto", 4),
         ("staged", (12, 11, 13), 2, 1, "c128", "staged", 16)]


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02456_amd.solver import Solver
    return Solver


def _rel(a, b):
    a = a.to(torch.complex128)
    b = b.to(torch.complex128)
    return ((a - b).abs().max() / b.abs().max()).item()


@pytest.mark.parametrize("name,shape,R,batch,dtype,path,fixed", CASES)
def test_fixed_iteration_step_is_captured_and_replayed(name, shape, R, batch, dtype, path, fixed):
    Solver = _gpu()
    print("case: skyrme graph", name, shape, "R", R, "batch", batch, dtype, flush=True)
    h, dt = 0.3, 0.002
    kw = dict(radius=R, order="first", s1=1.0, batch=batch, dtype=dtype, path=path)
    s_fix = Solver(shape, h, dt, meanfield=dict(MF, fixed_iters=fixed), **kw)
    s_ada = Solver(shape, h, dt, meanfield=MF, **kw)
    expect = {"onepass-orbitals": "onepass", "two-stage-orbitals": "fused", "staged": "staged"}[name]
    assert s_fix.path == expect, s_fix.path
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    rdt = torch.float32 if dtype == "c64" else torch.float64
    full = shape + (batch,) if batch > 1 else shape
    psi0 = torch.from_numpy(W.random_complex(full, seed=21)).to(cdt).cuda().contiguous()
    V = torch.from_numpy(W.random_potential(shape, seed=22)).to(rdt).cuda().contiguous()
    # complex64 states: the FP32 bar for the state and for the FP64 aux it drives
    tol = TOL if dtype == "c128" else 1e-5

    # the fixed-iteration step against the adaptive one, eagerly
    pa, aa = psi0.clone(), s_ada.new_aux()
    pf, af = psi0.clone(), s_fix.new_aux()
    s_ada.step(pa, aa, V, 3)
    s_fix.step(pf, af, V, 3)
    torch.cuda.synchronize()
    assert _rel(pf, pa) < tol
    assert _rel(af, aa) < tol
    assert s_fix.potential_unconverged() == 0
    _, iy0, ic0 = s_fix.potential_iterations()
    assert iy0 >= 3 and ic0 >= 3

    # capture one step (the eager steps above built what the launches need)
    pg, ag = psi0.clone(), s_fix.new_aux()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s_fix.step(pg, ag, V, 1)
    pe, ae = psi0.clone(), s_ada.new_aux()
    pg.copy_(psi0)
    ag.zero_()
    torch.cuda.synchronize()
    for k in range(3):
        g.replay()
        s_ada.step(pe, ae, V, 1)
        torch.cuda.synchronize()
        err, aerr = _rel(pg, pe), _rel(ag, ae)
        print("  replay %d: psi %.2e aux %.2e" % (k, err, aerr), flush=True)
        assert err < tol and aerr < tol, (k, err, aerr)
        # the program's own eager work between the replays
        junk = torch.linspace(0, 1, 4096, device="cuda", dtype=torch.float64)
        assert abs(junk.sum().item() - 2048.0) < 1e-9
    assert s_fix.potential_unconverged() == 0
    _, iy1, ic1 = s_fix.potential_iterations()
    assert iy1 >= iy0 + 3 and ic1 >= ic0 + 3  # the replays' solves were tallied on the device


def test_capture_needs_fixed_iterations_and_built_descriptors():
    Solver = _gpu()
    from paper_1908_02456_amd._lib import AbcError
    shape, h, dt = (14, 12, 16), 0.3, 0.002
    print("case: skyrme graph refusals", shape, flush=True)
    psi = torch.from_numpy(W.random_complex(shape + (2,), seed=23)).cuda().contiguous()
    s = Solver(shape, h, dt, order="first", s1=1.0, batch=2, meanfield=MF)
    aux = s.new_aux()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(AbcError, match="pcg_fixed"):
        with torch.cuda.graph(g):
            s.step(psi, aux, None, 1)
    # fixed iterations, but the two-stage orbital launch has not been set up
    # for this potential and parity yet
    s2 = Solver(shape, h, dt, order="first", s1=1.0, batch=2, meanfield=dict(MF, fixed_iters=4))
    assert s2.path == "fused"
    aux2 = s2.new_aux()
    g2 = torch.cuda.CUDAGraph()
    with pytest.raises(AbcError, match="outside the capture"):
        with torch.cuda.graph(g2):
            s2.step(psi, aux2, None, 1)
    torch.cuda.synchronize()
