"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and the ctypes structure matches the C layout.  No GPU."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_1908_02456_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abc_dtn.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(abc_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    return _lib.load()


def test_header_declares_what_binding_uses():
    assert set(_declared_functions()) == set(_lib.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (\w+)", out))
    missing = [n for n in _declared_functions() if n not in exported]
    assert not missing, missing


def test_params_struct_layout_matches_c():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "abc_dtn.h"
int main(void) {
  printf("%zu", sizeof(abc_params));
#define F(x) printf(" %zu", offsetof(abc_params, x));
  F(nx) F(ny) F(nz) F(h) F(dt) F(radius) F(order) F(form) F(s0) F(s1) F(s2) F(window) F(fejer)
  F(dtype) F(batch) F(meanfield) F(t0) F(t3) F(path) F(diag_every) F(reserved) F(s3) F(s4) F(v0) F(a_yukawa) F(e2)
  F(pcg_tol) F(pcg_maxit) F(pcg_fixed) F(reserved2)
  printf("\n");
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I" + os.path.dirname(HEADER), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    P = _lib.AbcParams
    names = ["nx", "ny", "nz", "h", "dt", "radius", "order", "form", "s0", "s1", "s2", "window", "fejer",
             "dtype", "batch", "meanfield", "t0", "t3", "path", "diag_every", "reserved", "s3", "s4", "v0", "a_yukawa",
             "e2",
             "pcg_tol", "pcg_maxit", "pcg_fixed", "reserved2"]
    assert vals[0] == ctypes.sizeof(P)
    assert vals[1:] == [getattr(P, n).offset for n in names]


def test_defaults_and_error_text(lib):
    p = _lib.AbcParams()
    lib.abc_params_default(ctypes.byref(p))
    assert (p.radius, p.order, p.form, p.dtype, p.batch, p.fejer) == (1, 3, 1, 0, 1, 1)
    assert (p.s0, p.s1, p.s2, p.s3, p.s4) == (1.0, 1.0, 0.0, 3.0, 10.0)
    assert (p.v0, p.a_yukawa, p.e2, p.pcg_tol, p.pcg_maxit) == (0.0, 1.0, 0.0, 1e-12, 1000)
    # invalid parameters are rejected before any device call
    p.radius = 7
    ctx = ctypes.c_void_p()
    st = lib.abc_setup(ctypes.byref(p), ctypes.byref(ctx))
    assert st == _lib.ABC_EINVAL
    assert b"radius" in lib.abc_last_error()
    assert not ctx.value
    lib.abc_params_default(ctypes.byref(p))
    p.s1 = -1.0
    assert lib.abc_setup(ctypes.byref(p), ctypes.byref(ctx)) == _lib.ABC_EUNSTABLE
    lib.abc_params_default(ctypes.byref(p))
    p.reserved[0] = 1
    assert lib.abc_setup(ctypes.byref(p), ctypes.byref(ctx)) == _lib.ABC_EINVAL
    lib.abc_destroy(None)


BAD_PARAMS = [
    (dict(nx=0), _lib.ABC_EINVAL, b"positive"),
    (dict(radius=0), _lib.ABC_EINVAL, b"radius"),
    (dict(radius=3, nx=6), _lib.ABC_EINVAL, b"2R+1"),
    (dict(h=0.0), _lib.ABC_EINVAL, b"h and dt"),
    (dict(dt=float("nan")), _lib.ABC_EINVAL, b"h and dt"),
    (dict(order=9), _lib.ABC_EINVAL, b"order"),
    (dict(form=5), _lib.ABC_EINVAL, b"form"),
    (dict(dtype=3), _lib.ABC_EINVAL, b"dtype"),
    (dict(batch=0), _lib.ABC_EINVAL, b"batch"),
    (dict(meanfield=4), _lib.ABC_EINVAL, b"mean field"),
    (dict(path=7), _lib.ABC_EINVAL, b"path"),
    (dict(window=-1), _lib.ABC_EINVAL, b"window"),
    (dict(diag_every=-1), _lib.ABC_EINVAL, b"diag_every"),
    (dict(order=2, s0=0.0), _lib.ABC_EUNSTABLE, b"s0"),
    (dict(order=3, s1=-1.0), _lib.ABC_EUNSTABLE, b"s1"),
    (dict(order=3, form=1, s2=2.0), _lib.ABC_ENOTSUP, b"face form"),
    (dict(order=5), _lib.ABC_EINVAL, b"order"),
    (dict(order=4, form=0, s2=2.0, s3=2.0), _lib.ABC_EINVAL, b"distinct"),
    (dict(order=4, form=0, s2=0.0), _lib.ABC_EINVAL, b"positive"),
    (dict(order=4, form=0, s2=2.0, s4=float("inf")), _lib.ABC_EINVAL, b"positive"),
    (dict(order=4, form=1, s2=2.0), _lib.ABC_ENOTSUP, b"box form only"),
    (dict(meanfield=3), _lib.ABC_EINVAL, b"mean field"),
    (dict(meanfield=2, v0=1.0, a_yukawa=0.0), _lib.ABC_EINVAL, b"Yukawa range"),
    (dict(meanfield=2, pcg_tol=0.0), _lib.ABC_EINVAL, b"pcg_tol"),
    (dict(meanfield=2, pcg_maxit=0), _lib.ABC_EINVAL, b"pcg_maxit"),
    (dict(meanfield=2, pcg_fixed=-1), _lib.ABC_EINVAL, b"pcg_fixed"),
    (dict(meanfield=2, e2=float("nan")), _lib.ABC_EINVAL, b"finite"),
]


@pytest.mark.parametrize("changes,status,text", BAD_PARAMS)
def test_setup_rejects_invalid_parameters(lib, changes, status, text):
    # every rule of the parameter check fires before any device call
    p = _lib.AbcParams()
    lib.abc_params_default(ctypes.byref(p))
    p.nx = p.ny = p.nz = 8
    p.h, p.dt = 0.25, 0.004
    for k, v in changes.items():
        setattr(p, k, v)
    ctx = ctypes.c_void_p()
    assert lib.abc_setup(ctypes.byref(p), ctypes.byref(ctx)) == status
    assert text in lib.abc_last_error()
    assert not ctx.value


def test_reserved_fields_must_be_zero(lib):
    p = _lib.AbcParams()
    lib.abc_params_default(ctypes.byref(p))
    p.nx = p.ny = p.nz = 8
    p.h, p.dt = 0.25, 0.004
    p.reserved[1] = 1
    ctx = ctypes.c_void_p()
    assert lib.abc_setup(ctypes.byref(p), ctypes.byref(ctx)) == _lib.ABC_EINVAL
    assert b"reserved" in lib.abc_last_error()
    p.reserved[1] = 0
    p.reserved2[1] = 1
    assert lib.abc_setup(ctypes.byref(p), ctypes.byref(ctx)) == _lib.ABC_EINVAL
    assert b"reserved" in lib.abc_last_error()


def test_h2_objective_rejects_invalid_arguments_without_a_device(lib):
    p = _lib.AbcParams()
    lib.abc_params_default(ctypes.byref(p))
    p.nx = p.ny = p.nz = 8
    pts = (ctypes.c_double * 2)(1.0, 2.0)
    out = (ctypes.c_double * 2)()
    assert lib.abc_h2_objective(None, pts, 2, 16, 64, out, None) == _lib.ABC_EINVAL
    assert lib.abc_h2_objective(ctypes.byref(p), pts, 0, 16, 64, out, None) == _lib.ABC_EINVAL
    assert lib.abc_h2_objective(ctypes.byref(p), pts, 2, 2, 64, out, None) == _lib.ABC_EINVAL
    assert lib.abc_h2_objective(ctypes.byref(p), pts, 2, 16, 8, out, None) == _lib.ABC_EINVAL
    bad = (ctypes.c_double * 2)(1.0, -2.0)
    assert lib.abc_h2_objective(ctypes.byref(p), bad, 2, 16, 64, out, None) == _lib.ABC_EINVAL
    assert b"positive" in lib.abc_last_error()
    p.order = 2
    assert lib.abc_h2_objective(ctypes.byref(p), pts, 2, 16, 64, out, None) == _lib.ABC_ENOTSUP
    p.order, p.radius = 3, 2
    assert lib.abc_h2_objective(ctypes.byref(p), pts, 2, 16, 64, out, None) == _lib.ABC_ENOTSUP
    assert b"R = 1" in lib.abc_last_error()


def test_null_arguments_are_rejected_without_a_device(lib):
    vp = ctypes.c_void_p
    assert lib.abc_effective_potential(None, None, None, None, None) == _lib.ABC_EINVAL
    assert lib.abc_state_save(None, None, None, 0, b"/tmp/x", None) == _lib.ABC_EINVAL
    assert lib.abc_state_load(None, None, None, None, b"/tmp/x", None) == _lib.ABC_EINVAL
    assert lib.abc_potential_iterations(None, None) == _lib.ABC_EINVAL
    assert lib.abc_setup(None, None) == _lib.ABC_EINVAL
    assert lib.abc_step(None, None, None, None, 1, None) == _lib.ABC_EINVAL
    k = ctypes.c_int(0)
    assert lib.abc_step_timed(None, None, None, None, 1, None, None, 0, ctypes.byref(k)) == _lib.ABC_EINVAL
    J = ctypes.c_double(0)
    assert lib.abc_adjoint(None, None, None, 1, 0, 0, None, None, ctypes.byref(J), None) == _lib.ABC_EINVAL
    assert lib.abc_diagnostics(None, None, None, None, None, None) == _lib.ABC_EINVAL
    assert lib.abc_diagnostics_noalloc(None, None, None, None, None, None) == _lib.ABC_EINVAL
    assert lib.abc_step_monitored(None, None, None, None, 1, None, None, 1, None) == _lib.ABC_EINVAL
    assert lib.abc_export(None, 0, None, 0) == _lib.ABC_EINVAL
    assert lib.abc_tune(None, None, None, None, None, None) == _lib.ABC_EINVAL
    b = vp()
    assert lib.abc_setup_batch(None, 0, ctypes.byref(b)) == _lib.ABC_EINVAL
    assert lib.abc_step_batch(None, None, None, None, 1, 0, None) == _lib.ABC_EINVAL
    assert lib.abc_tune_batch(None, None, None, None, None) == _lib.ABC_EINVAL
    assert lib.abc_aux_elems(None) == 0 and lib.abc_device_bytes(None) == 0
    assert lib.abc_batch_aux_elems(None, 0) == 0 and lib.abc_batch_launch_groups(None) == 0
    assert lib.abc_batch_tile_depth(None, 0) == 0
    assert lib.abc_launch_label(None, 0) is None
    lib.abc_destroy(None)
    lib.abc_destroy_batch(None)
