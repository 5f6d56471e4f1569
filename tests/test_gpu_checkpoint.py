"""Checkpoint and resume through the C ABI: a run interrupted by a save and a
load continues bit for bit; mismatched contexts and unreadable files are
rejected."""
import os
import tempfile

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1908_02456_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02456_amd.solver import Solver
    return Solver


@pytest.mark.parametrize("kw", [dict(order="first", window=0), dict(order="first", window=2, batch=3),
                                dict(order="zeroth", dtype="c64"),
                                dict(order="second", form="box", s_points=(1.0, 2.0, 3.0, 10.0))])
def test_resume_is_bit_identical(kw):
    print("case: checkpoint", kw, flush=True)
    Solver = _gpu()
    shape = (12, 10, 11) if kw.get("form") != "box" else (6, 6, 6)
    s = Solver(shape, 0.3, 0.004, **kw)
    cdt = torch.complex64 if kw.get("dtype") == "c64" else torch.complex128
    full = s.psi_shape()
    psi = torch.from_numpy(W.random_complex(full, seed=3)).to(cdt).cuda().contiguous()
    aux = s.new_aux()
    s.step(psi, aux, None, 5)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "state.bin")
        s.save_state(path, psi, aux, step=5)
        s.step(psi, aux, None, 4)
        ref_psi, ref_aux = psi.clone(), aux.clone()
        psi2 = torch.zeros_like(psi)
        aux2 = torch.zeros_like(aux)
        assert s.load_state(path, psi2, aux2) == 5
        s.step(psi2, aux2, None, 4)
        assert torch.equal(psi2, ref_psi) and torch.equal(aux2, ref_aux)
        # a context with another box, dtype or order refuses the file
        from paper_1908_02456_amd._lib import AbcError
        other = Solver((shape[0] + 1,) + shape[1:], 0.3, 0.004, **kw)
        with pytest.raises(AbcError, match="does not match"):
            other.load_state(path, torch.zeros(other.psi_shape(), dtype=cdt, device="cuda"), other.new_aux())
    with pytest.raises(AbcError, match="ABC_EIO"):
        s.load_state("/nonexistent/dir/state.bin", psi2, aux2)
