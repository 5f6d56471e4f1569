"""abc_diagnostics_noalloc (reduction partials in the library's fixed device
array) against abc_diagnostics (partials in the context's scratch), through
the C ABI: two calls in a row, the second on a smaller input, each output
bit-identical to the existing entry point's (same kernels, same fixed-order
reduction).  Also: a batch beyond the array's capacity is refused before any
work is queued."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1908_02456_amd import _lib, workloads as W  # noqa: E402
from paper_1908_02456_amd.solver import Solver  # noqa: E402

pytestmark = pytest.mark.gpu


def _both(s, psi, aux, V):
    lib = _lib.load()
    n = 3 * s.batch + 1
    a = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    b = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    ap = aux.data_ptr() if aux is not None else None
    vp = V.data_ptr() if V is not None else None
    stream = torch.cuda.current_stream().cuda_stream
    _lib.check(lib.abc_diagnostics(s._ctx, psi.data_ptr(), ap, vp, a.data_ptr(), stream))
    _lib.check(lib.abc_diagnostics_noalloc(s._ctx, psi.data_ptr(), ap, vp, b.data_ptr(), stream))
    torch.cuda.synchronize()
    return a.cpu(), b.cpu()


def test_noalloc_diagnostics_match_context_scratch_twice():
    # first call: 3 orbitals, first order with a filled aux, t0/t3 mean field
    shape = (20, 19, 18)
    s1 = Solver(shape, 0.25, 0.004, order="first", s1=1.0, window=1, batch=3, meanfield=(-1.0, 0.5))
    psi1 = torch.from_numpy(W.random_complex(shape + (3,), seed=11)).cuda()
    V1 = torch.from_numpy(W.random_potential(shape, seed=12)).cuda()
    aux1 = s1.new_aux()
    s1.step(psi1, aux1, V1, 3)          # non-zero aux, so W differs from N
    a, b = _both(s1, psi1, aux1, V1)
    assert torch.isfinite(a).all()
    assert torch.equal(a, b)
    assert not torch.equal(a[3:6], a[0:3])      # W includes f^* Q f
    # second call, smaller: one orbital, zeroth order, complex64, no V
    shape2 = (9, 10, 11)
    s2 = Solver(shape2, 0.25, 0.004, order="zeroth", s0=1.0, dtype="c64")
    psi2 = torch.from_numpy(W.random_complex(shape2, seed=13)).to(torch.complex64).cuda()
    a2, b2 = _both(s2, psi2, None, None)
    assert torch.isfinite(a2).all()
    assert torch.equal(a2, b2)
    # the norm matches a direct sum (independent of both entry points)
    h3 = 0.25 ** 3
    ref = h3 * float(np.sum(np.abs(psi2.cpu().numpy().astype(np.complex128)) ** 2))
    assert abs(b2[0].item() - ref) <= 1e-12 * ref


def test_noalloc_diagnostics_refuse_a_batch_beyond_the_fixed_array():
    lib = _lib.load()
    shape = (4, 4, 4)
    s = Solver(shape, 0.25, 0.004, order="dirichlet", batch=65)
    psi = torch.zeros(shape + (65,), dtype=torch.complex128, device="cuda")
    out = torch.zeros(3 * 65 + 1, dtype=torch.float64, device="cuda")
    st = lib.abc_diagnostics_noalloc(s._ctx, psi.data_ptr(), None, None, out.data_ptr(), None)
    assert st == _lib.ABC_EINVAL
    assert b"64 orbitals" in lib.abc_last_error()
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
