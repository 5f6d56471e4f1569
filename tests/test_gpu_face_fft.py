"""Exact face sections applied by zero-padded 2D FFTs (face form, no taper,
window >= n - 1) against the oracle's direct Toeplitz sections.

The transforms round at about eps log2(P) of the largest values, so the
FP64 bar of 1e-12 relative to the state's maximum applies unchanged (FP32
stencil: 1e-5)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import integrate
from paper_1908_02456_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02456_amd.solver import Solver
    return Solver


CASES = [
    ((10, 10, 10), 1, "first", 1, "c128", 4),
    ((9, 12, 11), 1, "zeroth", 1, "c128", 4),
    ((11, 10, 12), 2, "first", 1, "c128", 3),
    ((9, 9, 9), 2, "zeroth", 1, "c128", 3),
    ((12, 11, 10), 1, "first", 3, "c128", 3),
    ((10, 11, 12), 1, "first", 1, "c64", 4),
    ((24, 26, 25), 1, "first", 1, "c128", 3),
    ((9, 10, 11), 3, "first", 1, "c128", 3),
    ((10, 9, 11), 3, "zeroth", 2, "c128", 3),
    ((6, 70, 68), 1, "first", 1, "c128", 2),  # 256-point transforms on the z faces
]


@pytest.mark.parametrize("shape,R,order,batch,dtype,steps", CASES)
def test_exact_section_by_fft_matches_oracle(shape, R, order, batch, dtype, steps):
    print("case: face fft", shape, R, order, batch, dtype, steps, flush=True)
    Solver = _gpu()
    h, dt, w = 0.25, 0.004, max(shape) - 1
    full = shape if batch == 1 else shape + (batch,)
    psi0 = W.random_complex(full, seed=21)
    V = W.random_potential(shape, seed=22, scale=2.0)
    st = integrate.make_setup(shape, h, dt, R, order, s0=1.5, s1=1.5, window=w, use_window=False)
    ref_psi, ref_aux, _ = integrate.run(st, psi0, V, steps)
    s = Solver(shape, h, dt, radius=R, order=order, s0=1.5, s1=1.5, window=w, fejer=False, batch=batch, dtype=dtype)
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    rdt = torch.float64 if dtype == "c128" else torch.float32
    psi = torch.from_numpy(psi0).to(cdt).cuda().contiguous()
    aux = s.new_aux()
    s.step(psi, aux, torch.from_numpy(V).to(rdt).cuda(), steps)
    got = psi.cpu().numpy().astype(np.complex128)
    err = np.abs(got - ref_psi).max() / np.abs(ref_psi).max()
    tol = 1e-12 if dtype == "c128" else 1e-5
    print("  err %.2e" % err, flush=True)
    assert err < tol, err
    if order == "first":
        ref_flat = integrate.pack_aux(st, ref_aux)
        ga = aux.cpu().numpy()[:ref_flat.size]
        aerr = np.abs(ga - ref_flat).max() / np.abs(ref_flat).max()
        assert aerr < (1e-12 if dtype == "c128" else 1e-5), aerr


def test_fft_plan_only_for_exact_sections():
    # the padded work and spectra buffers exist with the exact section (no
    # taper, window >= n - 1) and not with a tapered or narrower window
    Solver = _gpu()
    shape = (12, 12, 12)
    b_exact = Solver(shape, 0.25, 0.004, window=11, fejer=False).device_bytes()
    b_taper = Solver(shape, 0.25, 0.004, window=11, fejer=True).device_bytes()
    b_narrow = Solver(shape, 0.25, 0.004, window=10, fejer=False).device_bytes()
    # 3 face pairs x (two 2 x 32 x 32 work slabs + one spectrum) complex128
    assert b_exact - b_taper > 200000 and b_exact - b_narrow > 200000, (b_exact, b_taper, b_narrow)
