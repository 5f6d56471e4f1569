"""The absorbing run against the large zero-boundary box, on the device and in
the oracle: the relative L2 errors that bench.py reports for the headline
(at 128^3 against 256^3) are computed here the same way at a size the
oracle runs in seconds, and must agree with the oracle's figures."""
import sys
import os

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

torch = pytest.importorskip("torch")

from test_oracle_face_halfspace import large_box_errors  # noqa: E402
from paper_1908_02456_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def device_large_box_errors(n=10, big=30, h=0.25, dt=0.005, steps=150, windows=(0, 3)):
    from paper_1908_02456_amd.solver import Solver
    psi0 = W.gaussian_packet((n,) * 3, h, center=(0.3, 0.0, 0.0), k=(3.0, 0.0, 0.0))
    off = (big - n) // 2
    pb = torch.zeros((big,) * 3, dtype=torch.complex128, device="cuda")
    pb[off:off + n, off:off + n, off:off + n] = torch.from_numpy(psi0)
    Solver((big,) * 3, h, dt, order="dirichlet").step(pb, None, None, steps)
    ref = pb[off:off + n, off:off + n, off:off + n].clone()
    nr = torch.linalg.vector_norm(ref).item()
    out = {}
    p = torch.from_numpy(psi0).cuda()
    Solver((n,) * 3, h, dt, order="dirichlet").step(p, None, None, steps)
    out["dirichlet"] = torch.linalg.vector_norm(p - ref).item() / nr
    for w in windows:
        s = Solver((n,) * 3, h, dt, order="first", s1=1.0, window=w)
        p = torch.from_numpy(psi0).cuda()
        s.step(p, s.new_aux(), None, steps)
        out["first_w%d" % w] = torch.linalg.vector_norm(p - ref).item() / nr
    torch.cuda.synchronize()
    return out


def test_large_box_errors_match_oracle():
    dev = device_large_box_errors()
    ref = large_box_errors()
    for k in ref:
        assert abs(dev[k] - ref[k]) <= 1e-10 * ref[k], (k, dev[k], ref[k])
    assert dev["first_w3"] < dev["first_w0"] < dev["dirichlet"]
