"""Pins of the oracle's second-order condition (Sec. 3.3): four-point
interpolation of the DtN map, the first-order rewriting of the dynamics
against the paper's second-derivative form, and the absorption ordering the
paper reports (no GPU)."""
import numpy as np
import pytest

from oracle import dtn, integrate
from paper_1908_02456_amd import workloads as W

S_PTS = (1.0, 2.0, 3.0, 10.0)


def test_second_order_interpolates_the_dtn_map_at_four_points():
    shape, h = (6, 6, 7), 0.3
    bo = dtn.box_second(shape, h, 1, S_PTS)
    for s in S_PTS:
        K = dtn.dtn_box(shape, h, 1, s)
        assert np.abs(dtn.r22(bo.B1, bo.B0, bo.A1, bo.A0, s) - K).max() < 1e-12 * np.abs(K).max()
    # and is an approximation, not an identity, elsewhere
    K5 = dtn.dtn_box(shape, h, 1, 5.0)
    assert np.abs(dtn.r22(bo.B1, bo.B0, bo.A1, bo.A0, 5.0) - K5).max() > 1e-6 * np.abs(K5).max()


def test_face_symbols_interpolate_mode_by_mode():
    h, R = 0.25, 2
    fo = dtn.face_second(h, R, S_PTS, 1, P=64)
    sym = fo.symbol
    for s in S_PTS:
        k = dtn.face_symbol_k(s, h, R, 64)
        for (i, j) in [(0, 0), (5, 17), (40, 3)]:
            lhs = (s * s * np.eye(R) - s * sym["b1"][i, j] - sym["b0"][i, j]) @ k[i, j]
            rhs = s * sym["a1"][i, j] + (sym["c"][i, j] - sym["b1"][i, j] @ sym["a1"][i, j])
            assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(rhs).max()


def test_first_order_rewriting_matches_the_second_derivative_form():
    # with g = df/dt - A1 E psi the generator must reproduce
    # d2f/dt2 = B1 df/dt + B0 f + A1 E dpsi/dt + A0 E psi for any state
    shape, h = (6, 7, 6), 0.3
    st = integrate.make_setup(shape, h, 0.01, 1, "second", form="box", s_second=S_PTS)
    bo = st.box
    psi = W.random_complex(shape, seed=5) - (0.5 + 0.5j)
    n = len(bo.gamma)
    rng = np.random.default_rng(6)
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    g = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    V = W.random_potential(shape, seed=7)
    dpsi, (df, dg) = integrate.generator(st, psi, (f, g), V)
    _, (ddf, _) = integrate.generator(st, dpsi, (df, dg), V)
    Eps = psi[bo.gamma[:, 0], bo.gamma[:, 1], bo.gamma[:, 2]]
    Edps = dpsi[bo.gamma[:, 0], bo.gamma[:, 1], bo.gamma[:, 2]]
    want = bo.B1 @ df + bo.B0 @ f + bo.A1 @ Edps + bo.A0 @ Eps
    assert np.abs(ddf - want).max() < 1e-10 * np.abs(want).max()


@pytest.mark.slow
def test_second_order_absorbs_better_than_first_order():
    # free packet leaving a 12^3 box: error against a 28^3 Dirichlet box
    # (same h, dt, data zero-extended) orders as the paper reports
    n, big, h, dt, steps = 12, 28, 0.25, 0.005, 160
    psi0 = W.gaussian_packet((n,) * 3, h, k=(2.0, 0.0, 0.0))
    V = np.zeros((n,) * 3)
    off = (big - n) // 2
    pb = np.zeros((big,) * 3, complex)
    pb[off:off + n, off:off + n, off:off + n] = psi0
    ref, _, _ = integrate.run(integrate.make_setup((big,) * 3, h, dt, 1, "dirichlet"), pb, np.zeros((big,) * 3), steps)
    ref = ref[off:off + n, off:off + n, off:off + n]

    def err(order, **kw):
        st = integrate.make_setup((n,) * 3, h, dt, 1, order, form="box", **kw)
        psi, _, _ = integrate.run(st, psi0, V, steps)
        return np.linalg.norm(psi - ref) / np.linalg.norm(ref)

    e_dir, e1, e2 = err("dirichlet"), err("first", s1=1.0), err("second", s_second=S_PTS)
    assert e2 < 0.5 * e1 < 0.5 * e_dir, (e_dir, e1, e2)


# R >= 2: the interpolation in the dominant subspace of the four maps
REDUCED_CASES = [((7, 7, 7), 2, 0.3), ((7, 8, 7), 2, 0.3), ((9, 9, 9), 3, 0.3)]


def _stack_singular_values(Ks):
    G = sum((K @ K.conj().T).real for K in Ks)
    w = np.sort(np.linalg.eigvalsh(G))[::-1]
    return np.sqrt(np.maximum(w, 0.0) / w[0])


@pytest.mark.parametrize("shape,R,h", REDUCED_CASES)
def test_second_order_subspace_is_the_outer_layer_past_a_gap(shape, R, h):
    # the kept dimension is the number of points of the outermost boundary
    # layer, and the cut falls in a gap at least ten times wide on either
    # side of tau (so that any eigen-solver keeps the same subspace)
    Ks = [dtn.dtn_box(shape, h, R, s) for s in S_PTS]
    U = dtn.dominant_subspace(Ks)
    nz, ny, nx = shape
    assert U.shape[1] == nx * ny * nz - (nx - 2) * (ny - 2) * (nz - 2)
    sv = _stack_singular_values(Ks)
    r = U.shape[1]
    assert sv[r - 1] > 5 * dtn.SECOND_ORDER_TAU and sv[r] < dtn.SECOND_ORDER_TAU / 5, (sv[r - 1], sv[r])
    assert np.abs(U.T @ U - np.eye(r)).max() < 1e-12
    # nothing is dropped at R = 1
    K1 = [dtn.dtn_box((6, 6, 7), 0.3, 1, s) for s in S_PTS]
    assert dtn.dominant_subspace(K1).shape[1] == K1[0].shape[0]


@pytest.mark.parametrize("shape,R,h", REDUCED_CASES[::2])
def test_second_order_reduced_interpolation(shape, R, h):
    Ks = [dtn.dtn_box(shape, h, R, s) for s in S_PTS]
    bo = dtn.box_second(shape, h, R, S_PTS)
    U = dtn.dominant_subspace(Ks)
    n, r = U.shape
    P = U @ U.T
    for K, s in zip(Ks, S_PTS):
        # R22 interpolates the map's part on the subspace at the four points
        assert np.abs(dtn.r22(bo.B1, bo.B0, bo.A1, bo.A0, s) - P @ K @ P).max() < 1e-9 * np.abs(K).max()
        # and what is left out is the small part, below tau of the map
        assert np.linalg.norm(K - P @ K @ P, 2) < dtn.SECOND_ORDER_TAU * np.linalg.norm(K, 2)
    # every coefficient maps span(U) into itself and is zero off it
    Q = np.eye(n) - P
    for X in (bo.B1, bo.B0, bo.A1, bo.A0):
        assert np.abs(Q @ X).max() < 1e-11 * np.abs(X).max() and np.abs(X @ Q).max() < 1e-11 * np.abs(X).max()
    # the result does not depend on the basis of the subspace
    rot, _ = np.linalg.qr(np.random.default_rng(11).standard_normal((r, r)))
    V = U @ rot
    alt = dtn.interp_second([V.T @ K @ V for K in Ks], S_PTS)
    for X, Y in zip((bo.B1, bo.B0, bo.A1, bo.A0), alt):
        assert np.abs(V @ Y @ V.T - X).max() < 1e-7 * np.abs(X).max()
    # the reduced auxiliary dynamics [[0, I], [B0, B1]] is stable
    red = [U.T @ X @ U for X in (bo.B1, bo.B0)]
    G = np.block([[np.zeros((r, r)), np.eye(r)], [red[1], red[0]]])
    assert np.linalg.eigvals(G).real.max() < 0


@pytest.mark.slow
def test_second_order_absorbs_better_than_first_order_R2():
    # the same ordering with the wider stencil, where the coefficients come
    # from the dominant subspace
    n, big, h, dt, steps, R = 10, 26, 0.25, 0.004, 160, 2
    psi0 = W.gaussian_packet((n,) * 3, h, k=(2.0, 0.0, 0.0))
    V = np.zeros((n,) * 3)
    off = (big - n) // 2
    pb = np.zeros((big,) * 3, complex)
    pb[off:off + n, off:off + n, off:off + n] = psi0
    ref, _, _ = integrate.run(integrate.make_setup((big,) * 3, h, dt, R, "dirichlet"), pb, np.zeros((big,) * 3),
                              steps)
    ref = ref[off:off + n, off:off + n, off:off + n]

    def err(order, **kw):
        st = integrate.make_setup((n,) * 3, h, dt, R, order, form="box", **kw)
        psi, _, _ = integrate.run(st, psi0, V, steps)
        return np.linalg.norm(psi - ref) / np.linalg.norm(ref)

    e_dir, e1, e2 = err("dirichlet"), err("first", s1=1.0), err("second", s_second=S_PTS)
    assert e2 < 0.5 * e1 < 0.5 * e_dir, (e_dir, e1, e2)
