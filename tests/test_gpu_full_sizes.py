"""Two workloads at their full sizes against the FP64 oracle.

* The TDHF batch: 32 seeded oscillator orbitals on 96^3 with the mean field
  U = t0 rho + t3 rho^2 (t0 = -1, t3 = 0.5) rebuilt every step, first order
  (w = 0): two steps on the device (complex64 on the one-pass orbital sweep,
  complex128 on the two-stage orbital kernels), every element against the
  oracle's two steps (1e-5 and 1e-12 of the largest magnitude).
* The uneven batch: the 64 boxes of the workload (N in {48, 64, 96, 128,
  160}, zeroth and first order mixed) stepped together, one step from
  seeded random data, sampled at 12 points per box against oracle sub-box
  steps (a point's value after one step depends only on what lies within 4
  of it; see the maximum-size tests).
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import integrate  # noqa: E402
from paper_1908_02456_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
REACH = 4


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02456_amd.solver import Solver, Batch
    return Solver, Batch


@pytest.fixture(scope="module")
def tdhf_reference():
    n, nb, h, dt, steps = 96, 32, 0.2, 0.002, 2
    orb = W.oscillator_orbitals((n,) * 3, h, nb, seed=3)
    st = integrate.make_setup((n,) * 3, h, dt, 1, "first", form="faces", s1=1.0, window=0, t0=-1.0, t3=0.5)
    ref, ref_aux, _ = integrate.run(st, orb, np.zeros((n,) * 3), steps)
    return dict(n=n, nb=nb, h=h, dt=dt, steps=steps, orb=orb, ref=ref,
                ref_flat=integrate.pack_aux(st, ref_aux))


@pytest.mark.parametrize("dtype,path", [("c64", "onepass"), ("c128", "fused")])
def test_tdhf_batch_full_size_matches_oracle(tdhf_reference, dtype, path):
    Solver, _ = _gpu()
    r = tdhf_reference
    print("case: TDHF 96^3 x 32", dtype, flush=True)
    s = Solver((r["n"],) * 3, r["h"], r["dt"], order="first", s1=1.0, window=0, dtype=dtype, batch=r["nb"],
               meanfield=(-1.0, 0.5))
    assert s.path == path, s.path
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    psi = torch.from_numpy(r["orb"]).to(cdt).cuda().contiguous()
    aux = s.new_aux()
    s.step(psi, aux, None, r["steps"])
    torch.cuda.synchronize()
    got = psi.cpu().numpy().astype(np.complex128)
    err = np.abs(got - r["ref"]).max() / np.abs(r["ref"]).max()
    ga = aux.cpu().numpy()[:r["ref_flat"].size]
    aerr = np.abs(ga - r["ref_flat"]).max() / np.abs(r["ref_flat"]).max()
    print("  psi %.2e aux %.2e" % (err, aerr), flush=True)
    tol = 1e-5 if dtype == "c64" else 1e-12
    assert err < tol and aerr < tol, (err, aerr)


def _samples(shape, rng):
    nz, ny, nx = shape
    pts = [(0, 0, 0), (nz - 1, ny - 1, nx - 1)]
    for d in (0, 2):
        for axis in range(3):
            p = [int(rng.integers(0, n)) for n in shape]
            p[axis] = d if rng.random() < 0.5 else shape[axis] - 1 - d
            pts.append(tuple(p))
    for _ in range(4):
        pts.append(tuple(int(rng.integers(REACH + 1, n - REACH - 1)) for n in shape))
    return pts


def test_uneven_batch_full_size_sampled_against_oracle():
    Solver, Batch = _gpu()
    print("case: 64-instance batch, sampled", flush=True)
    insts = W.uneven_batch()
    cfgs = [dict(shape=d["shape"], h=d["h"], dt=d["dt"], order=d["order"], s0=d["s0"], s1=d["s1"], window=0)
            for d in insts]
    b = Batch(cfgs)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(77)
    psis, Vs = [], []
    for d in insts:
        re = torch.randn(d["shape"], dtype=torch.float64, device="cuda", generator=gen)
        im = torch.randn(d["shape"], dtype=torch.float64, device="cuda", generator=gen)
        psis.append(torch.complex(re, im).contiguous())
        Vs.append((3.0 * torch.rand(d["shape"], dtype=torch.float64, device="cuda", generator=gen)).contiguous())
    auxs = [b.new_aux(i) for i in range(len(insts))]
    rng = np.random.default_rng(8)
    work = []
    for i, d in enumerate(insts):
        for p in _samples(d["shape"], rng):
            lo = [max(0, c - REACH) for c in p]
            hi = [min(n - 1, c + REACH) for c, n in zip(p, d["shape"])]
            sl = tuple(slice(a, c + 1) for a, c in zip(lo, hi))
            work.append((i, p, lo, psis[i][sl].cpu().numpy(), Vs[i][sl].cpu().numpy()))
    b.step(psis, auxs, Vs, 1)
    torch.cuda.synchronize()
    setups = {}
    worst = 0.0
    for i, p, lo, psub, vsub in work:
        d = insts[i]
        key = (psub.shape, d["order"])
        if key not in setups:
            setups[key] = integrate.make_setup(psub.shape, d["h"], d["dt"], 1, d["order"], form="faces",
                                               s0=d["s0"], s1=d["s1"], window=0)
        ref, _, _ = integrate.run(setups[key], psub, vsub, 1)
        r = ref[tuple(c - l for c, l in zip(p, lo))]
        g = psis[i][p].item()
        worst = max(worst, abs(g - r) / max(abs(r), 1.0))
    print("  %d points over %d boxes, max error %.2e (relative to max(|value|, 1))" % (len(work), len(insts), worst),
          flush=True)
    assert worst < 1e-12, worst
