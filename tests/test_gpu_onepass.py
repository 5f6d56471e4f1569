"""The one-pass sweep (all four stages of a Taylor-4 step in one z-marching
launch, the step polynomial applied as the product of its two real
quadratic factors) against the FP64 oracle, element by element: complex128
at 1e-12 and complex64 at 1e-5 of the largest magnitude, the first order's
auxiliary values at 1e-12 (they stay FP64) and 1e-5.  Boxes span several
tiles in y and z with ragged tails (complex128 tiles are 4 rows by 16
planes, complex64 tiles 8 by 8), including a last tile one row or one plane
deep, whose face row or plane then lies in the previous tile's halo; narrow,
odd and full 128-column rows; odd and even step counts (the ping-pong ends
in the caller's buffers either way).  Also: the full 128^3 headline workload
agrees with the two-pass fused path, every point compared; and the first
order with a windowed or exact face operator (the condition-free sweep plus
the boundary-shell rounds) against the oracle on the same boxes and against
the staged path at 128^3."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from test_gpu_parity import TOL32, TOL64, _run_pair  # noqa: E402
from paper_1908_02456_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

SHAPES = [(21, 19, 37), (35, 9, 128), (7, 6, 5), (18, 33, 100)]


@pytest.mark.parametrize("order", ["dirichlet", "zeroth"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("steps", [3, 4])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_onepass_parity(order, shape, steps, dtype):
    r = _run_pair("onepass %s %s" % (order, dtype), shape, 0.25, 0.004, 1, order, steps, dtype=dtype,
                  path="onepass", seed=7)
    tol = TOL64 if dtype == "c128" else TOL32
    assert r["err"] <= tol, r["err"]


# first order: ny > rows per tile (12 / 16) and nz > planes per tile + 4
# (20 / 12), so that a tile meets at most one y-face row and one z-face plane
FIRST_SHAPES = [(21, 19, 37), (33, 17, 128), (24, 33, 100), (22, 18, 9)]


@pytest.mark.parametrize("shape", FIRST_SHAPES)
@pytest.mark.parametrize("steps", [3, 4])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_onepass_first_order_parity(shape, steps, dtype):
    r = _run_pair("onepass first %s" % dtype, shape, 0.25, 0.004, 1, "first", steps, s1=1.5, dtype=dtype,
                  path="onepass", seed=11)
    tol = TOL64 if dtype == "c128" else TOL32
    assert r["err"] <= tol, r["err"]
    assert r["aux_err"] <= tol, r["aux_err"]


@pytest.mark.parametrize("order", ["dirichlet", "first"])
def test_onepass_headline_size_matches_two_pass(order):
    from paper_1908_02456_amd.solver import Solver
    wl = W.well_packet(n=128)
    print("case: onepass 128^3 %s vs fused two-pass" % order, flush=True)
    out, aux = [], []
    for path in ("fused", "onepass"):
        s = Solver((128,) * 3, wl.h, wl.dt, order=order, s1=wl.s1, path=path)
        psi = torch.from_numpy(wl.psi0).cuda()
        a = s.new_aux()
        s.step(psi, a, torch.from_numpy(wl.V).cuda(), 7)
        out.append(psi)
        aux.append(a)
    torch.cuda.synchronize()
    d = (out[0] - out[1]).abs().max().item() / out[0].abs().max().item()
    assert d <= TOL64, d
    if order == "first":
        da = (aux[0] - aux[1]).abs().max().item() / aux[0].abs().max().item()
        assert da <= TOL64, da


def test_onepass_refuses_what_it_does_not_cover():
    from paper_1908_02456_amd.solver import Solver
    from paper_1908_02456_amd._lib import AbcError
    with pytest.raises(AbcError):
        Solver((10, 10, 130), 0.25, 0.004, order="dirichlet", path="onepass")
    with pytest.raises(AbcError):
        Solver((10, 10, 10), 0.25, 0.004, order="dirichlet", radius=2, path="onepass")


# first order with a non-local face operator: the condition-free sweep plus
# the boundary-shell rounds (window 1: per-element face kernel; 3: tiled;
# exact sections: zero-padded FFTs)
SHELL_CASES = [(1, True), (3, True), (None, False)]


@pytest.mark.parametrize("window,fejer", SHELL_CASES, ids=["w1", "w3", "exact"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("steps", [3, 4])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_onepass_windowed_first_order_parity(window, fejer, shape, steps, dtype):
    w = max(shape) - 1 if window is None else window
    r = _run_pair("onepass shell first w=%d %s" % (w, dtype), shape, 0.25, 0.004, 1, "first", steps, s1=1.5,
                  window=w, fejer=fejer, dtype=dtype, path="onepass", seed=13)
    assert r["solver"].path == "onepass"
    tol = TOL64 if dtype == "c128" else TOL32
    assert r["err"] <= tol, r["err"]
    assert r["aux_err"] <= tol, r["aux_err"]


@pytest.mark.parametrize("window,fejer", [(8, True), (127, False)], ids=["w8", "exact"])
def test_onepass_windowed_headline_size_matches_staged(window, fejer):
    from paper_1908_02456_amd.solver import Solver
    wl = W.well_packet(n=128)
    print("case: onepass shell 128^3 first w=%d vs staged" % window, flush=True)
    out, aux = [], []
    for path in ("auto", "onepass"):
        s = Solver((128,) * 3, wl.h, wl.dt, order="first", s1=wl.s1, window=window, fejer=fejer, path=path)
        assert s.path == ("staged" if path == "auto" else "onepass")
        psi = torch.from_numpy(wl.psi0).cuda()
        a = s.new_aux()
        s.step(psi, a, torch.from_numpy(wl.V).cuda(), 7)
        out.append(psi)
        aux.append(a)
    torch.cuda.synchronize()
    d = (out[0] - out[1]).abs().max().item() / out[0].abs().max().item()
    assert d <= TOL64, d
    da = (aux[0] - aux[1]).abs().max().item() / aux[0].abs().max().item()
    assert da <= TOL64, da


# orbital batches (orbital-innermost state, transposed once per call) on the
# one-pass sweep: one launch per step over all orbitals (blockIdx.y), the
# mean field rebuilt from the current state before every step
@pytest.mark.parametrize("order", ["first", "zeroth", "dirichlet"])
@pytest.mark.parametrize("meanfield", [None, (-1.0, 0.5)], ids=["plain", "meanfield"])
@pytest.mark.parametrize("steps", [3, 4])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_onepass_orbital_batch_parity(order, meanfield, steps, dtype):
    r = _run_pair("onepass orbitals %s %s" % (order, dtype), (21, 19, 37), 0.25, 0.004, 1, order, steps, s0=1.5,
                  s1=1.5, batch=3, meanfield=meanfield, dtype=dtype, path="onepass", seed=17)
    assert r["solver"].path == "onepass"
    tol = TOL64 if dtype == "c128" else TOL32
    assert r["err"] <= tol, r["err"]
    if order == "first":
        assert r["aux_err"] <= tol, r["aux_err"]


def test_onepass_orbital_batch_long_range_meanfield_matches_two_pass():
    from paper_1908_02456_amd.solver import Solver
    print("case: onepass orbitals with the long-range mean field", flush=True)
    shape, nb = (22, 18, 30), 4
    mf = dict(t0=-1.0, t3=0.5, v0=-2.0, a=0.7, e2=1.44, tol=1e-13, maxit=500)
    psi0 = torch.from_numpy(W.random_complex(shape + (nb,), seed=21)).cuda() * 0.3
    V = torch.from_numpy(W.random_potential(shape, seed=22, scale=2.0)).cuda()
    out, aux = [], []
    for path in ("fused", "onepass"):
        s = Solver(shape, 0.25, 0.004, order="first", s1=1.5, batch=nb, meanfield=mf, path=path)
        assert s.path == path
        psi = psi0.clone()
        a = s.new_aux()
        s.step(psi, a, V, 5)
        out.append(psi)
        aux.append(a)
    torch.cuda.synchronize()
    d = (out[0] - out[1]).abs().max().item() / out[0].abs().max().item()
    assert d <= TOL64, d
    da = (aux[0] - aux[1]).abs().max().item() / max(aux[0].abs().max().item(), 1e-300)
    assert da <= TOL64, da
