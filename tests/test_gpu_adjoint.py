"""HIP adjoint vs the oracle's FP64 adjoint (same seeded inputs, element by
element) and vs central finite differences of the HIP forward map through
the torch.autograd binding.  Tolerance: 1e-12 relative to the largest entry
for the oracle comparison (complex128 on both sides)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adjoint as oadj, integrate
from paper_1908_02456_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _solver_cls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02456_amd.solver import Solver
    return Solver


CASES = [
    ("dirichlet-prob", dict(order="dirichlet"), 1, "prob", 0),
    ("periodic-energy", dict(order="periodic"), 2, "energy", 3),
    ("zeroth-R2-w1", dict(order="zeroth", s0=1.5, window=1), 2, "prob", 1),
    ("zeroth-R1-w0-energy", dict(order="zeroth", s0=2.0, window=0), 1, "energy", 0),
    ("first-w0-prob", dict(order="first", s1=1.5, window=0), 1, "prob", 0),
    ("first-w0-energy", dict(order="first", s1=1.0, window=0), 1, "energy", 2),
    ("first-w2-prob", dict(order="first", s1=1.0, window=2), 1, "prob", 100),
    ("first-w1-nofejer", dict(order="first", s1=1.0, window=1, fejer=False), 1, "prob", 4),
]


@pytest.mark.parametrize("name,kw,R,kind,stride", CASES)
def test_adjoint_matches_oracle(name, kw, R, kind, stride):
    print("case: adjoint", name, "stride", stride, flush=True)
    Solver = _solver_cls()
    shape, h, dt, steps = (9, 10, 11), 0.3, 0.01, 7
    psi0 = W.random_complex(shape, seed=31) - (0.5 + 0.5j)
    V = W.random_potential(shape, seed=32, scale=2.0)
    okw = dict(kw)
    fejer = okw.pop("fejer", True)
    st = integrate.make_setup(shape, h, dt, R, use_window=fejer, **okw)
    J, gpsi, gV = oadj.adjoint_run(st, psi0, V, steps, kind)
    s = Solver(shape, h, dt, radius=R, fejer=fejer, path="staged", **okw)
    Jg, gpsi_g, gV_g = s.adjoint(torch.from_numpy(psi0).cuda(), torch.from_numpy(V).cuda(), steps, kind, stride)
    gpsi_g, gV_g = gpsi_g.cpu().numpy(), gV_g.cpu().numpy()
    assert abs(Jg - J) < TOL * abs(J), (Jg, J)
    assert np.abs(gpsi_g - gpsi).max() < TOL * np.abs(gpsi).max()
    assert np.abs(gV_g - gV).max() < TOL * np.abs(gV).max()


FUSED_CASES = [c for c in CASES if c[0] in ("dirichlet-prob", "zeroth-R1-w0-energy", "first-w0-prob",
                                             "first-w0-energy")]


@pytest.mark.parametrize("name,kw,R,kind,stride0", FUSED_CASES)
@pytest.mark.parametrize("stride", [0, 1, 3, 7])
def test_adjoint_with_fused_recompute_matches_oracle(name, kw, R, kind, stride0, stride):
    # the two-stage fused kernels recompute the segments, keeping the Horner
    # intermediates u1, u2, u3 of every step, and the potential gradient is
    # formed from them (stride 7 = the whole run as one segment: no separate
    # forward sweep)
    print("case: adjoint fused recompute", name, "stride", stride, flush=True)
    Solver = _solver_cls()
    shape, h, dt, steps = (9, 10, 11), 0.3, 0.01, 7
    psi0 = W.random_complex(shape, seed=31) - (0.5 + 0.5j)
    V = W.random_potential(shape, seed=32, scale=2.0)
    okw = dict(kw)
    st = integrate.make_setup(shape, h, dt, R, **okw)
    J, gpsi, gV = oadj.adjoint_run(st, psi0, V, steps, kind)
    s = Solver(shape, h, dt, radius=R, path="fused", **okw)
    assert s.path == "fused"
    Jg, gpsi_g, gV_g = s.adjoint(torch.from_numpy(psi0).cuda(), torch.from_numpy(V).cuda(), steps, kind, stride)
    gpsi_g, gV_g = gpsi_g.cpu().numpy(), gV_g.cpu().numpy()
    assert abs(Jg - J) < TOL * abs(J), (Jg, J)
    assert np.abs(gpsi_g - gpsi).max() < TOL * np.abs(gpsi).max()
    # dJ/dV sums per step terms dt Im(conj(y_j) u_j) of size about dt |lambda|
    # |psi|; the device evaluates the adjoint step in Horner form, the oracle
    # as the Taylor sum, so they differ by the terms' rounding.  Where J is
    # conserved (the probability in a box with zero boundary values) the
    # terms cancel to a gradient a hundred times smaller than they are, and
    # the bar is set on the terms' size.
    terms = dt * np.abs(gpsi).max() * np.abs(psi0).max()
    assert np.abs(gV_g - gV).max() < TOL * max(np.abs(gV).max(), terms)


def test_adjoint_zero_steps_and_strides_agree():
    print("case: adjoint strides", flush=True)
    Solver = _solver_cls()
    shape = (12, 11, 10)
    psi0 = torch.from_numpy(W.random_complex(shape, seed=41)).cuda()
    V = torch.from_numpy(W.random_potential(shape, seed=42)).cuda()
    s = Solver(shape, 0.25, 0.004, order="first", s1=1.0, window=0)
    J0, g0, gV0 = s.adjoint(psi0, V, 0, "prob")
    assert torch.allclose(g0, 2 * 0.25 ** 3 * psi0, rtol=0, atol=0) and float(gV0.abs().max()) == 0.0
    # checkpoints come from the forward sweep (fused path) and segment states
    # from the recompute, so strides agree to rounding, not bit for bit
    outs = [s.adjoint(psi0, V, 13, "prob", st) for st in (1, 4, 0, 13, 50)]
    for J, g, gV in outs[1:]:
        assert J == outs[0][0]
        assert float((g - outs[0][1]).abs().max()) < 1e-12 * float(outs[0][1].abs().max())
        assert float((gV - outs[0][2]).abs().max()) < 1e-12 * float(outs[0][2].abs().max())


def test_adjoint_rejects_unsupported():
    print("case: adjoint unsupported", flush=True)
    Solver = _solver_cls()
    from paper_1908_02456_amd._lib import AbcError, ABC_ENOTSUP
    shape = (8, 8, 8)
    psi0 = torch.zeros(shape, dtype=torch.complex64, device="cuda")
    with pytest.raises(AbcError) as e:
        Solver(shape, 0.3, 0.004, order="first", dtype="c64").adjoint(psi0, None, 2)
    assert e.value.status == ABC_ENOTSUP
    psi0 = psi0.to(torch.complex128)
    for kw in (dict(order="first", radius=2), dict(order="zeroth", form="box")):
        with pytest.raises(AbcError) as e:
            Solver(shape, 0.3, 0.004, **kw).adjoint(psi0, None, 2)
        assert e.value.status == ABC_ENOTSUP


def _fields(prm, a, c, k, dev):
    n, h = prm["n"], prm["h"]
    Z, Y, X = (torch.from_numpy(v).to(dev) for v in W.mesh((n, n, n), h))
    V = -a * torch.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / 2)
    x0 = prm["packet_center"]
    env = torch.exp(-((X - x0[0]) ** 2 + (Y - x0[1]) ** 2 + (Z - x0[2]) ** 2) / 2)
    phase = k[0] * X + k[1] * Y + k[2] * Z
    psi0 = torch.complex(env * torch.cos(phase), env * torch.sin(phase))
    return V, psi0


def _check_parameter_gradients(prm, eps, rtol):
    Solver = _solver_cls()
    from paper_1908_02456_amd.autograd import abc_objective
    dev = torch.device("cuda")
    n = prm["n"]
    s = Solver((n, n, n), prm["h"], prm["dt"], order="first", s1=prm["s1"], window=prm["window"], path="staged")
    a = torch.tensor(prm["amplitude"], dtype=torch.float64, device=dev, requires_grad=True)
    c = torch.tensor(prm["well_center"], dtype=torch.float64, device=dev, requires_grad=True)
    k = torch.tensor(prm["k"], dtype=torch.float64, device=dev, requires_grad=True)
    V, psi0 = _fields(prm, a, c, k, dev)
    J = abc_objective(s, psi0, V, prm["steps"], "prob")
    J.backward()
    grads = {"a": a.grad.item(), "c_x": c.grad[0].item(), "c_y": c.grad[1].item(), "k_x": k.grad[0].item(),
             "k_z": k.grad[2].item()}

    def forward(da=0.0, dc=(0, 0, 0), dk=(0, 0, 0)):
        with torch.no_grad():
            Vp, pp = _fields(prm, a + da, c + torch.tensor(dc, device=dev), k + torch.tensor(dk, device=dev), dev)
            pp = pp.contiguous()
            aux = s.new_aux()
            s.step(pp, aux, Vp.contiguous(), prm["steps"])
            torch.cuda.synchronize()
            return prm["h"] ** 3 * float((pp.abs() ** 2).sum())

    # the objective's value equals a plain forward run
    assert abs(J.item() - forward()) < 1e-12 * J.item()
    fds = {"a": (forward(da=eps) - forward(da=-eps)) / (2 * eps),
           "c_x": (forward(dc=(eps, 0, 0)) - forward(dc=(-eps, 0, 0))) / (2 * eps),
           "c_y": (forward(dc=(0, eps, 0)) - forward(dc=(0, -eps, 0))) / (2 * eps),
           "k_x": (forward(dk=(eps, 0, 0)) - forward(dk=(-eps, 0, 0))) / (2 * eps),
           "k_z": (forward(dk=(0, 0, eps)) - forward(dk=(0, 0, -eps))) / (2 * eps)}
    scale = max(abs(v) for v in grads.values())
    for name in grads:
        print(name, grads[name], fds[name], flush=True)
        assert abs(grads[name] - fds[name]) < rtol * scale, (name, grads[name], fds[name])


def test_autograd_parameter_gradients_small():
    print("case: autograd 32^3", flush=True)
    prm = W.adjoint_packet(n=32, steps=60)
    prm["packet_center"] = (1.0, 0.0, 0.0)
    _check_parameter_gradients(prm, 1e-4, 1e-6)


def test_autograd_parameter_gradients_full_size():
    # 96^3, 500 steps, first order, FP64, sqrt(n) checkpointing
    print("case: autograd 96^3 x 500", flush=True)
    _check_parameter_gradients(W.adjoint_packet(), 1e-4, 1e-6)


@pytest.mark.parametrize("objective", ["prob", "energy"])
def test_objective_without_gradients_skips_the_reverse_sweep(objective, monkeypatch):
    print("case: objective without gradients", objective, flush=True)
    Solver = _solver_cls()
    from paper_1908_02456_amd.autograd import abc_objective
    shape, h, dt, steps = (12, 11, 10), 0.25, 0.004, 9
    s = Solver(shape, h, dt, order="first", s1=1.5, window=1, path="staged")
    psi0 = torch.from_numpy(W.random_complex(shape, seed=5)).cuda()
    V = torch.from_numpy(W.random_potential(shape, seed=6, scale=2.0)).cuda()
    J_adj, _, _ = s.adjoint(psi0, V, steps, objective)
    calls = []
    monkeypatch.setattr(s, "adjoint", lambda *a, **k: calls.append(1))
    J = abc_objective(s, psi0, V, steps, objective)
    assert not calls
    assert not J.requires_grad
    assert abs(J.item() - J_adj) <= 1e-12 * abs(J_adj)
