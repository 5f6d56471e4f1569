"""H2 objective of the first-order interpolation point (Sec. 5 proposal; face
form, R = 1) on the device against the FP64 oracle.

Tolerance: J is a sum of P^2 N positive terms whose inputs agree with the
oracle's to rounding, except the kernel of B, which the host setups of the
two sides build independently (the face-kernel export agrees at 1e-12 of its
largest coefficient).  1e-10 relative leaves room for that kernel difference
to move J; the measured agreement is printed.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import h2

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02456_amd import solver
    return solver


@pytest.mark.parametrize("h,w,fejer,P,N,pts", [
    (0.2, 0, True, 32, 1024, (0.5, 3.0, 60.0)),
    (0.25, 2, True, 16, 512, (1.0, 40.0)),
    (0.2, 3, False, 16, 768, (2.0, 150.0)),
    (0.3, 1, True, 24, 333, (0.05, 7.0)),
])
def test_h2_objective_matches_oracle(h, w, fejer, P, N, pts):
    print("case: h2", h, w, fejer, P, N, pts, flush=True)
    api = _api()
    got = api.h2_objective(h, pts, window=w, fejer=fejer, modes=P, nodes=N)
    for s1, g in zip(pts, got):
        ref = h2.h2_objective(h, s1, w, P=P, N=N, window=fejer)
        print("  s1 %g: rel diff %.2e" % (s1, abs(g - ref) / ref), flush=True)
        assert abs(g - ref) < TOL * ref, (s1, g, ref)


def test_optimal_point_is_a_minimum_of_the_oracle_objective():
    api = _api()
    h, P, N = 0.2, 16, 512
    s_best, j_best = api.optimal_point(h, window=0, modes=P, nodes=N)
    print("case: h2 optimum s1 = %.6g, J = %.6e" % (s_best, j_best), flush=True)
    ref = h2.h2_objective(h, s_best, 0, P=P, N=N)
    assert abs(ref - j_best) < TOL * ref
    for f in (0.9, 1.1):
        assert ref <= h2.h2_objective(h, s_best * f, 0, P=P, N=N)
    # and no grid point does better
    xs = np.exp(np.linspace(math.log(1e-2), math.log(1e4), 25))
    assert j_best <= api.h2_objective(h, xs, window=0, modes=P, nodes=N).min()


def test_h2_objective_rejects_other_orders():
    api = _api()
    from paper_1908_02456_amd._lib import AbcError
    import ctypes
    from paper_1908_02456_amd import _lib
    lib = _lib.load()
    p = api.make_params((8, 8, 8), 0.2, 1e-3, order="zeroth", form="faces")
    pts = np.array([1.0])
    out = np.zeros(1)
    st = lib.abc_h2_objective(ctypes.byref(p), pts.ctypes.data, 1, 16, 64, out.ctypes.data, None)
    assert st == _lib.ABC_ENOTSUP
    with pytest.raises(AbcError):
        _lib.check(st)
