"""The largest boxes each path accepts, against the FP64 oracle on sampled
points.

The one-pass and two-stage sweeps address the state with 32-bit byte
offsets, so they accept states below 4 GiB (128 x 1440 x 1440 at complex128,
128 x 2040 x 2040 at complex64); a larger state (128 x 1500 x 1500,
complex128) runs on the staged path, whose indices are 64-bit.  One step of
the first-order condition (face form, w = 0) from seeded random data.

Sampled parity: after one Taylor-4 step (four stages of a radius-1 stencil)
a point depends only on the data within 4 of it and on the boundary
variables of faces within that distance, which start at zero.  So the
oracle steps a sub-box reaching 4 beyond the sample point (clipped at the
box), with the real faces where it is clipped and zero outside elsewhere;
the spurious edges of the sub-box reach at most 3 points in, and the sample
point's value is exact.  Samples: random interior points, points at depth
0 to 3 from each face, on edges and at the eight corners."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import integrate

pytestmark = pytest.mark.gpu

H, DT, S1 = 0.2, 0.002, 1.0
REACH = 4  # four stages of a radius-1 stencil


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02456_amd.solver import Solver
    return Solver


def _samples(shape, rng, n_interior=16):
    nz, ny, nx = shape
    pts = [(z, y, x) for z in (0, nz - 1) for y in (0, ny - 1) for x in (0, nx - 1)]  # corners
    for d in range(4):  # depth 0 .. 3 from each face, elsewhere random
        for axis in range(3):
            for side in (0, 1):
                p = [int(rng.integers(0, n)) for n in shape]
                p[axis] = d if side == 0 else shape[axis] - 1 - d
                pts.append(tuple(p))
    for _ in range(4):  # on edges
        p = [int(rng.integers(0, n)) for n in shape]
        a, b = rng.choice(3, size=2, replace=False)
        p[a] = 0 if rng.random() < 0.5 else shape[a] - 1
        p[b] = 0 if rng.random() < 0.5 else shape[b] - 1
        pts.append(tuple(p))
    for _ in range(n_interior):
        pts.append(tuple(int(rng.integers(REACH + 1, n - REACH - 1)) for n in shape))
    return pts


def _check(shape, dtype, path_expect, path="auto", seed=0):
    Solver = _gpu()
    print("case: max size", shape, dtype, path, flush=True)
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    rdt = torch.float64 if dtype == "c128" else torch.float32
    s = Solver(shape, H, DT, order="first", s1=S1, dtype=dtype, path=path)
    assert s.path == path_expect, s.path
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1000 + seed)
    psi = torch.randn(shape, dtype=torch.float64, device="cuda", generator=gen).to(rdt)
    psi = torch.complex(psi, torch.randn(shape, dtype=torch.float64, device="cuda", generator=gen).to(rdt))
    assert psi.dtype == cdt
    V = (2.0 * torch.rand(shape, dtype=torch.float64, device="cuda", generator=gen)).to(rdt)
    rng = np.random.default_rng(seed)
    pts = _samples(shape, rng)
    # the sub-box data before the step
    subs = []
    for p in pts:
        lo = [max(0, c - REACH) for c in p]
        hi = [min(n - 1, c + REACH) for c, n in zip(p, shape)]
        sl = tuple(slice(a, b + 1) for a, b in zip(lo, hi))
        subs.append((p, lo, psi[sl].cpu().numpy().astype(np.complex128), V[sl].cpu().numpy().astype(np.float64)))
    aux = s.new_aux()
    s.step(psi, aux, V, 1)
    torch.cuda.synchronize()
    got = [psi[p].item() for p in pts]
    del psi, V, aux, s
    torch.cuda.empty_cache()
    setups = {}
    worst, scale = 0.0, 0.0
    for (p, lo, psub, vsub), g in zip(subs, got):
        key = psub.shape
        if key not in setups:
            setups[key] = integrate.make_setup(key, H, DT, 1, "first", form="faces", s1=S1, window=0)
        ref, _, _ = integrate.run(setups[key], psub, vsub, 1)
        r = ref[tuple(c - l for c, l in zip(p, lo))]
        worst = max(worst, abs(complex(g) - r))
        scale = max(scale, abs(r))
    err = worst / scale
    print("  %d points, max relative error %.2e" % (len(pts), err), flush=True)
    assert err < (1e-12 if dtype == "c128" else 1e-5), err


def test_onepass_largest_state_c128():
    # 128 x 1440 x 1440 complex128: 3.97 GB, the largest below the 4 GiB limit
    _check((1440, 1440, 128), "c128", "onepass")


def test_two_stage_largest_state_c128():
    _check((1440, 1440, 128), "c128", "fused", path="fused", seed=1)


def test_onepass_largest_state_c64():
    # 128 x 2040 x 2040 complex64: 4.26 GB, 533 M points
    _check((2040, 2040, 128), "c64", "onepass", seed=2)


def test_state_beyond_4gib_runs_staged():
    # 128 x 1500 x 1500 complex128 (4.6 GB): the sweeps refuse it, the staged
    # path takes it with 64-bit indices
    _check((1500, 1500, 128), "c128", "staged", seed=3)
