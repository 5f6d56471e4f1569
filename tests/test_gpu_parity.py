"""HIP path vs the FP64 oracle, element by element, on the same seeded inputs.

FP64 path: max |psi_gpu - psi_oracle| <= 1e-12 max |psi_oracle| (and the same
for the auxiliary variable).  FP32 stencil path (complex64 state, FP64
auxiliary recurrences): 1e-5.  Every case prints its name before it touches
the GPU.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dtn, integrate
from paper_1908_02456_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02456_amd.solver import Solver
    return Solver


def _run_pair(name, shape, h, dt, R, order, steps, *, form="faces", s0=1.0, s1=1.0, s2=math.inf, window=0,
              fejer=True, batch=None, meanfield=None, dtype="c128", seed=0, psi0=None, V=None, path="auto"):
    print("case:", name, shape, "R", R, order, form, "w", window, "batch", batch, dtype, flush=True)
    Solver = _gpu()
    if psi0 is None:
        full = shape if batch is None else shape + (batch,)
        psi0 = W.random_complex(full, seed=seed)
    if V is None:
        V = W.random_potential(shape, seed=seed + 100, scale=2.0)
    st = integrate.make_setup(shape, h, dt, R, order, form=form, s0=s0, s1=s1, s2=s2, window=window,
                              use_window=fejer, t0=None if meanfield is None else meanfield[0],
                              t3=0.0 if meanfield is None else meanfield[1])
    ref_psi, ref_aux, _ = integrate.run(st, psi0, V, steps)
    solver = Solver(shape, h, dt, radius=R, order=order, form=form, s0=s0, s1=s1,
                    s2=(0.0 if math.isinf(s2) else s2), window=window, fejer=fejer, dtype=dtype,
                    batch=1 if batch is None else batch, meanfield=meanfield, path=path)
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    rdt = torch.float64 if dtype == "c128" else torch.float32
    psi = torch.from_numpy(psi0).to(cdt).cuda().contiguous()
    Vt = torch.from_numpy(V).to(rdt).cuda().contiguous()
    aux = solver.new_aux()
    solver.step(psi, aux, Vt, steps)
    torch.cuda.synchronize()
    got = psi.cpu().numpy().astype(np.complex128)
    scale = np.abs(ref_psi).max()
    err = np.abs(got - ref_psi).max() / scale
    out = {"err": err, "solver": solver, "psi": psi, "aux": aux, "V": Vt, "ref_psi": ref_psi,
           "ref_aux": ref_aux, "st": st}
    if order == "first":
        ref_flat = integrate.pack_aux(st, ref_aux)
        got_aux = aux.cpu().numpy()[:ref_flat.size]
        out["aux_err"] = np.abs(got_aux - ref_flat).max() / max(np.abs(ref_flat).max(), 1e-300)
    return out


@pytest.mark.parametrize("R", [1, 2, 3])
@pytest.mark.parametrize("order", ["dirichlet", "periodic"])
def test_no_condition_parity(R, order):
    r = _run_pair("plain", (13, 11, 17), 0.3, 0.01, R, order, 4, path="staged")
    assert r["err"] < TOL64, r["err"]


@pytest.mark.parametrize("R,window,fejer", [(1, 0, True), (1, 2, True), (2, 1, True), (3, 0, True),
                                            (1, 3, False)])
def test_zeroth_faces_parity(R, window, fejer):
    r = _run_pair("zeroth-faces", (12, 10, 14), 0.25, 0.004, R, "zeroth", 5, s0=2.0, window=window, fejer=fejer,
                  path="staged")
    assert r["err"] < TOL64, r["err"]


@pytest.mark.parametrize("R,window,fejer", [(1, 0, True), (1, 3, True), (2, 2, True), (3, 1, True),
                                            (1, 9, False)])
def test_first_faces_parity(R, window, fejer):
    r = _run_pair("first-faces", (11, 10, 13), 0.25, 0.004, R, "first", 6, s1=1.5, window=window, fejer=fejer,
                  path="staged")
    assert r["err"] < TOL64, r["err"]
    assert r["aux_err"] < TOL64, r["aux_err"]


def test_first_faces_full_section_parity():
    # window = n - 1 without taper: the exact Toeplitz section of each face
    r = _run_pair("first-faces-full", (10, 10, 10), 0.25, 0.004, 1, "first", 4, s1=1.0, window=9, fejer=False)
    assert r["err"] < TOL64 and r["aux_err"] < TOL64, (r["err"], r["aux_err"])


@pytest.mark.parametrize("R,order,s2", [(1, "zeroth", math.inf), (1, "first", math.inf), (1, "first", 2.0),
                                        (2, "zeroth", math.inf), (2, "first", math.inf)])
def test_box_form_parity(R, order, s2):
    n = 6 if R == 1 else 7
    r = _run_pair("box", (n, n, n), 0.3, 0.004, R, order, 5, form="box", s0=1.0, s1=1.0, s2=s2)
    assert r["err"] < TOL64, r["err"]
    if order == "first":
        assert r["aux_err"] < TOL64, r["aux_err"]


@pytest.mark.parametrize("shape,R,order,window", [((18, 21, 35), 1, "first", 3), ((19, 34, 17), 1, "zeroth", 4),
                                                  ((20, 19, 23), 2, "first", 2), ((17, 18, 33), 3, "zeroth", 2)])
def test_windowed_faces_several_tiles_parity(shape, R, order, window):
    # faces wider than one 16 x 16 tile of the LDS-tiled convolution, with
    # ragged tiles at the far edges
    r = _run_pair("faces-tiled", shape, 0.25, 0.004, R, order, 4, s0=1.5, s1=1.5, window=window)
    assert r["err"] < TOL64, r["err"]
    if order == "first":
        assert r["aux_err"] < TOL64, r["aux_err"]


@pytest.mark.parametrize("shape,R", [((35, 9, 70), 3), ((19, 7, 66), 2), ((17, 8, 64), 3), ((19, 9, 70), 1),
                                     ((9, 5, 130), 1)])
@pytest.mark.parametrize("order,window,dtype", [("dirichlet", 0, "c128"), ("zeroth", 0, "c128"),
                                                ("first", 0, "c128"), ("first", 2, "c128"), ("first", 0, "c64")])
def test_tiled_sweep_parity(shape, R, order, window, dtype):
    # one orbital on the staged path: the z-marching LDS-tiled stage sweep,
    # with several 64-column tiles in x, ragged row tiles in y and ragged
    # plane chunks in z (16 planes at R = 3, 8 at R = 1, 2); first order at
    # w = 0 runs it merged with the face work, the others as a launch of its
    # own
    r = _run_pair("tiled-sweep", shape, 0.25, 0.004, R, order, 3, s0=1.5, s1=1.5, window=window, dtype=dtype)
    tol = TOL64 if dtype == "c128" else TOL32
    assert r["err"] < tol, r["err"]
    if order == "first" and dtype == "c128":
        assert r["aux_err"] < TOL64, r["aux_err"]


@pytest.mark.parametrize("order", ["zeroth", "first"])
def test_box_form_large_operator_parity(order):
    # 28^3, R = 1: n_Gamma = 4376 rows, above the size where one orbital's
    # operator is applied with E y gathered once per stage and several rows
    # per workgroup (the small boxes above use one workgroup per row)
    n = 28
    print("case: box form large", order, flush=True)
    r = _run_pair("box-large", (n, n, n), 0.25, 0.004, 1, order, 3, form="box", s0=1.0, s1=1.0)
    assert r["err"] < TOL64, r["err"]
    if order == "first":
        assert r["aux_err"] < TOL64, r["aux_err"]


def test_batch_meanfield_parity():
    r = _run_pair("batch-meanfield", (9, 10, 11), 0.3, 0.004, 1, "first", 5, s1=1.0, window=2, batch=3,
                  meanfield=(-1.0, 0.5))
    assert r["err"] < TOL64 and r["aux_err"] < TOL64, (r["err"], r["aux_err"])


@pytest.mark.parametrize("R,window,dtype", [(2, 2, "c128"), (1, 3, "c128"), (3, 0, "c64")])
def test_single_orbital_meanfield_tiled_sweep_parity(R, window, dtype):
    # one orbital with the t0/t3 mean field on the staged path: the tiled
    # sweep reads the potential rebuilt from the current state every step
    r = _run_pair("meanfield-tiled", (13, 9, 70), 0.3, 0.004, R, "first", 4, s1=1.0, window=window,
                  meanfield=(-1.0, 0.5), dtype=dtype, path="staged")
    tol = TOL64 if dtype == "c128" else TOL32
    assert r["err"] < tol, r["err"]
    if dtype == "c128":
        assert r["aux_err"] < TOL64, r["aux_err"]


@pytest.mark.parametrize("order,window", [("first", 0), ("first", 2), ("zeroth", 1), ("dirichlet", 0)])
def test_fp32_path_parity(order, window):
    r = _run_pair("c64", (12, 11, 10), 0.25, 0.004, 1, order, 8, s0=1.0, s1=1.0, window=window, dtype="c64")
    assert r["err"] < TOL32, r["err"]


def test_face_kernel_export_matches_oracle():
    Solver = _gpu()
    h, R, w, s1 = 0.2, 2, 4, 1.3
    s = Solver((9, 9, 9), h, 0.002, radius=R, order="first", s1=s1, window=w, fejer=True)
    got = s.face_kernel()
    ref = dtn.face_first(h, R, s1, w).kernel
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_diagnostics_match_oracle():
    r = _run_pair("diag", (10, 9, 11), 0.25, 0.004, 1, "first", 3, s1=1.0, window=1)
    assert r["err"] < TOL64
    d = r["solver"].diagnostics(r["psi"], r["aux"], r["V"]).cpu().numpy()
    st = r["st"]
    ref = integrate.diagnostics(st, r["ref_psi"], r["ref_aux"], np.asarray(r["V"].cpu().numpy()))
    assert abs(d[0] - ref["norm"]) < 1e-12 * ref["norm"]
    assert abs(d[1] - ref["lyapunov"]) < 1e-12 * ref["lyapunov"]
    assert abs(d[2] - ref["energy"]) < 1e-11 * abs(ref["energy"])


def test_zero_steps_and_minimum_box():
    r = _run_pair("min-box", (3, 3, 3), 0.3, 0.004, 1, "first", 0, window=1)
    assert r["err"] == 0
    r = _run_pair("min-box", (3, 3, 3), 0.3, 0.004, 1, "first", 3, window=1)
    assert r["err"] < TOL64


@pytest.mark.parametrize("order", ["dirichlet", "zeroth", "first"])
@pytest.mark.parametrize("shape", [(21, 19, 37), (10, 17, 128), (16, 16, 16), (11, 12, 131), (6, 10, 250)])
@pytest.mark.parametrize("steps", [5, 6])
def test_fused_path_parity(order, shape, steps):
    # several 8x8 (y, z) tiles with ragged tails (10 = one plane/row past a
    # tile and a face row/plane in the halo); odd and even step counts; rows
    # of one x chunk (odd and even nx) and of several
    r = _run_pair("fused", shape, 0.25, 0.004, 1, order, steps, s0=1.5, s1=1.5, window=0, path="fused")
    assert r["solver"].use_fused
    assert r["err"] < TOL64, r["err"]
    if order == "first":
        assert r["aux_err"] < TOL64, r["aux_err"]


def _random_shapes(seed, count):
    # seeded box shapes for the fused path: ragged tiles in every direction,
    # rows of one or several x chunks, 4- and 8-plane tiles
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        out.append((int(rng.integers(6, 42)), int(rng.integers(10, 42)), int(rng.integers(4, 260))))
    return out


@pytest.mark.parametrize("order", ["dirichlet", "zeroth", "first"])
@pytest.mark.parametrize("shape", _random_shapes(1908, 6))
def test_fused_path_random_shapes(order, shape):
    r = _run_pair("fused-random", shape, 0.25, 0.004, 1, order, 3, s0=1.5, s1=1.5, window=0, path="fused",
                  seed=sum(shape))
    assert r["solver"].use_fused
    assert r["err"] < TOL64, r["err"]
    if order == "first":
        assert r["aux_err"] < TOL64, r["aux_err"]


@pytest.mark.parametrize("shape,dtype", [((17, 12, 20), "c128"), ((9, 10, 14), "c128"), ((17, 12, 20), "c64")])
def test_fused_first_order_face_plane_in_tile_halo(shape, dtype):
    # nz = 8k + 9 (8-plane tiles) and 4k + 5 (4-plane tiles): the last z-face
    # plane is a stage-1-only halo plane of one tile and an own plane of the
    # next; ny = 12 puts the last y-face row in the second tile's own rows
    r = _run_pair("fused-zhalo", shape, 0.25, 0.004, 1, "first", 5, s1=1.5, window=0, dtype=dtype, path="fused")
    assert r["solver"].use_fused
    tol = TOL64 if dtype == "c128" else TOL32
    assert r["err"] < tol, r["err"]
    if dtype == "c128":
        assert r["aux_err"] < TOL64, r["aux_err"]


@pytest.mark.parametrize("order", ["dirichlet", "zeroth", "first"])
@pytest.mark.parametrize("shape", [(19, 21, 45), (18, 20, 44)])
def test_fused_path_parity_fp32(order, shape):
    # odd and even row lengths (the x-face columns in the second or the
    # first column of a lane)
    r = _run_pair("fused-c64", shape, 0.25, 0.004, 1, order, 7, s1=1.0, window=0, dtype="c64",
                  path="fused")
    assert r["solver"].use_fused
    assert r["err"] < TOL32, r["err"]


def test_full_size_headline_parity():
    # the 128^3 single-orbital first-order workload in the launch
    # configuration the benchmark times, two steps, every grid point compared
    wl = W.well_packet(n=128)
    r = _run_pair("headline-128", (128, 128, 128), wl.h, wl.dt, 1, "first", 2, s1=wl.s1, window=0,
                  psi0=wl.psi0, V=wl.V, path="auto")
    assert r["solver"].use_fused
    assert r["err"] < TOL64, r["err"]
    assert r["aux_err"] < TOL64, r["aux_err"]


def test_staged_and_fused_agree():
    Solver = _gpu()
    shape = (24, 20, 40)
    psi0 = W.random_complex(shape, seed=11)
    V = W.random_potential(shape, seed=12)
    outs = []
    for path in ("staged", "fused"):
        s = Solver(shape, 0.25, 0.004, order="first", s1=2.0, window=0, path=path)
        psi = torch.from_numpy(psi0).cuda()
        aux = s.new_aux()
        s.step(psi, aux, torch.from_numpy(V).cuda(), 9)
        outs.append((psi.cpu().numpy(), aux.cpu().numpy()))
    scale = np.abs(outs[0][0]).max()
    assert np.abs(outs[0][0] - outs[1][0]).max() < 1e-12 * scale
    assert np.abs(outs[0][1] - outs[1][1]).max() < 1e-12 * np.abs(outs[0][1]).max()


def test_setup_rejects_unstable_dt():
    Solver = _gpu()
    from paper_1908_02456_amd._lib import AbcError, ABC_EUNSTABLE
    with pytest.raises(AbcError) as e:
        Solver((8, 8, 8), 0.1, 0.1, order="first")
    assert e.value.status == ABC_EUNSTABLE


@pytest.mark.parametrize("path,order", [("fused", "first"), ("staged", "first"), ("fused", "dirichlet")])
def test_step_timed_matches_step(path, order):
    # the measurement entry runs the same kernels with the same launch shapes
    print("case: step_timed", path, order, flush=True)
    Solver = _gpu()
    shape = (20, 18, 24)
    psi0 = W.random_complex(shape, seed=21)
    V = torch.from_numpy(W.random_potential(shape, seed=22)).cuda()
    outs = []
    for timed in (False, True):
        s = Solver(shape, 0.25, 0.004, order=order, s1=1.5, window=0, path=path)
        psi = torch.from_numpy(psi0).cuda()
        aux = s.new_aux()
        if timed:
            launches = s.step_timed(psi, aux, V, 5)
            assert launches and all(ms > 0 for _, ms in launches)
        else:
            s.step(psi, aux, V, 5)
        torch.cuda.synchronize()
        outs.append((psi.cpu().numpy(), aux.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_fused_first_order_small_box_falls_back():
    # the fused first-order kernel stages one y-face row and one z-face plane
    # per tile, so boxes with ny below 10 (or nz below 6) run on the staged path
    print("case: fused fallback", flush=True)
    Solver = _gpu()
    from paper_1908_02456_amd._lib import AbcError, ABC_ENOTSUP
    with pytest.raises(AbcError) as e:
        Solver((9, 8, 20), 0.25, 0.004, order="first", window=0, path="fused")
    assert e.value.status == ABC_ENOTSUP
    s = Solver((9, 8, 20), 0.25, 0.004, order="first", window=0, path="auto")
    assert not s.use_fused
    r = _run_pair("fused-fallback", (9, 8, 20), 0.25, 0.004, 1, "first", 4, s1=1.5, window=0, path="auto")
    assert r["err"] < TOL64 and r["aux_err"] < TOL64


@pytest.mark.parametrize("R,order,s2", [(1, "zeroth", math.inf), (1, "first", math.inf), (2, "first", math.inf),
                                        (1, "first", 2.0)])
def test_box_form_orbital_batch_parity(R, order, s2):
    # box form over an orbital batch: the operator is applied as one complex
    # GEMM per stage (FP64 matrix cores) instead of one matrix pass per orbital
    n = 6 if R == 1 else 7
    r = _run_pair("box-batch", (n, n, n), 0.3, 0.004, R, order, 5, form="box", s0=1.0, s1=1.0, s2=s2, batch=5)
    assert r["err"] < TOL64, r["err"]
    if order == "first":
        assert r["aux_err"] < TOL64, r["aux_err"]


@pytest.mark.parametrize("order,batch", [("first", 17), ("zeroth", 33), ("first", 64), ("zeroth", 2)])
def test_box_form_orbital_batch_gemm_tiles(order, batch):
    # the GEMM's ragged edges: n_Gamma = 7^3 - 5^3 = 218 operator rows (not a
    # multiple of the 16-row wave tile or the 64-row workgroup), K = 436 (first
    # order, [B | A]) or 218 (zeroth), both off the 16-wide k chunk, and 2, 17,
    # 33 or 64 orbitals (one to four 16-column tiles, ragged but the last)
    r = _run_pair("box-batch-gemm", (7, 7, 7), 0.3, 0.004, 1, order, 3, form="box", s0=1.0, s1=1.0,
                  batch=batch, seed=5)
    assert r["err"] < TOL64, r["err"]
    if order == "first":
        assert r["aux_err"] < TOL64, r["aux_err"]


def test_box_form_orbital_batch_over_64_is_refused():
    Solver = _gpu()
    from paper_1908_02456_amd._lib import AbcError
    with pytest.raises(AbcError):
        Solver((6, 6, 6), 0.3, 0.004, order="zeroth", form="box", batch=65)


@pytest.mark.parametrize("batch,meanfield,dtype,order", [(3, None, "c128", "first"), (5, (-1.0, 0.5), "c128", "first"),
                                                         (1, (-1.0, 0.5), "c128", "first"),
                                                         (4, (-1.0, 0.5), "c128", "zeroth"),
                                                         (6, (-1.0, 0.5), "c64", "first"),
                                                         (2, None, "c128", "dirichlet")])
@pytest.mark.parametrize("steps", [4, 5])
def test_orbital_batch_fused_parity(batch, meanfield, dtype, order, steps):
    # orbitals transposed to one array each and stepped as boxes of one
    # descriptor-driven launch, the mean field rebuilt before every step
    r = _run_pair("orbital-batch", (12, 11, 13), 0.25, 0.004, 1, order, steps, s0=1.5, s1=1.5, window=0,
                  batch=batch, meanfield=meanfield, dtype=dtype, path="fused")
    assert r["solver"].use_fused
    tol = TOL32 if dtype == "c64" else TOL64
    assert r["err"] < tol, r["err"]
    if order == "first":
        assert r["aux_err"] < (1e-5 if dtype == "c64" else TOL64), r["aux_err"]


def test_orbital_batch_fused_and_staged_agree():
    # 32 orbitals with the mean field, both paths on the same inputs
    print("case: orbital batch 32", flush=True)
    Solver = _gpu()
    shape, nb = (16, 14, 20), 32
    psi0 = W.random_complex(shape + (nb,), seed=61) * 0.3
    V = torch.from_numpy(W.random_potential(shape, seed=62)).cuda()
    outs = []
    for path in ("staged", "fused"):
        s = Solver(shape, 0.25, 0.004, order="first", s1=1.0, window=0, batch=nb, meanfield=(-1.0, 0.5), path=path)
        psi = torch.from_numpy(psi0).cuda()
        aux = s.new_aux()
        s.step(psi, aux, V, 7)
        torch.cuda.synchronize()
        outs.append((psi.cpu().numpy(), aux.cpu().numpy()))
    assert np.abs(outs[0][0] - outs[1][0]).max() < 1e-12 * np.abs(outs[0][0]).max()
    assert np.abs(outs[0][1] - outs[1][1]).max() < 1e-12 * np.abs(outs[0][1]).max()
