"""Pins of the oracle's interpolation (Section IV) against mathematics that
does not come from the oracle itself: polynomial exactness of the stencils,
a hand-worked example, and the tensor-product identity of per-level
interpolation built from independently derived Lagrange weights."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import fieldgen
from oracle import grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

EXACT_DEGREE = {"cubic": 3, "lquad": 2, "rquad": 2, "linear": 1, "copy": 0}


def test_golden_cubic_1d():
    g = json.load(open(os.path.join(GOLDEN, "stencil_cubic_1d.json")))
    x = np.array(g["x"], dtype=np.float64)
    assert grid.num_levels(x.shape) == g["levels"]
    (c,) = grid.decompose_level(x, (0,), "level", 3)
    assert c.tolist() == g["level0_coefficients_at_odd_indices"]


@pytest.mark.parametrize("n,L", [(1, 1), (2, 1), (3, 2), (5, 3), (8, 4), (9, 4), (64, 7), (65, 7), (66, 8),
                                 (512, 10), (513, 10), (1024, 11)])
def test_num_levels(n, L):
    assert grid.num_levels((n,)) == L
    # the coarsest level has one or two points
    assert 1 <= grid.compact_len(n, L - 1) <= 2


def _lagrange_weights(offsets, at=0):
    """Exact Lagrange weights for interpolating at ``at`` from points ``offsets``."""
    w = []
    for i, xi in enumerate(offsets):
        num, den = Fraction(1), Fraction(1)
        for j, xj in enumerate(offsets):
            if i != j:
                num *= at - xj
                den *= xi - xj
        w.append(num / den)
    return w


def _prolongation_1d(m, degree):
    """Dense (m x ceil(m/2)) 1D interpolation matrix, weights from Lagrange
    interpolation through the neighbours the rule allows (not from the oracle)."""
    mc = (m + 1) // 2
    S = np.zeros((m, mc), dtype=object)
    for i in range(m):
        if i % 2 == 0:
            S[i, i // 2] = Fraction(1)
            continue
        have = [o for o in (-3, -1, 1, 3) if 0 <= i + o <= m - 1]
        if 1 not in have:
            pts = [-1]
        elif degree == 1:
            pts = [-1, 1]
        elif -3 in have and 3 in have:
            pts = [-3, -1, 1, 3]
        elif 3 in have:
            pts = [-1, 1, 3]
        elif -3 in have:
            pts = [-3, -1, 1]
        else:
            pts = [-1, 1]
        for o, wgt in zip(pts, _lagrange_weights(pts)):
            S[i, (i + o) // 2] += wgt
    return S


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 7, 8, 9, 13, 16, 17])
@pytest.mark.parametrize("degree", [1, 3])
def test_stencil_matches_lagrange(m, degree):
    """The 1D stencil equals interpolation through its neighbours (checked
    on unit impulses)."""
    S = _prolongation_1d(m, degree)
    mc = (m + 1) // 2
    for k in range(mc):
        coarse = np.zeros(mc)
        coarse[k] = 1.0
        V = np.zeros(m)
        V[0::2] = coarse
        P = grid.predict_region(V, (0,), 0, degree)
        expect = [float(S[i, k]) for i in range(1, m, 2)]
        assert P.tolist() == expect


def _expected_zero(idx_odd_kind_degree, deg_poly):
    return EXACT_DEGREE[idx_odd_kind_degree] >= deg_poly


@pytest.mark.parametrize("kind", ["level", "region"])
@pytest.mark.parametrize("degree", [1, 3])
@pytest.mark.parametrize("shape", [(17,), (12, 13), (9, 10, 11), (16, 7, 12)])
@pytest.mark.parametrize("pdeg", [0, 1, 2, 3])
def test_polynomial_zero_coefficients(kind, degree, shape, pdeg):
    """A single-axis integer polynomial of degree pdeg gives exactly zero
    coefficients wherever the stencil along that axis is exact to pdeg, and
    a residual elsewhere (all arithmetic is exact: dyadic weights)."""
    d = len(shape)
    rng = np.random.default_rng(pdeg + 10 * d)
    for axis in range(d):
        coeffs = [[0] * 4 for _ in range(d)]
        for p in range(pdeg + 1):
            coeffs[axis][p] = int(rng.integers(1, 5)) * (1 if p % 2 == 0 else -1)
        x = fieldgen.polynomial_field(shape, coeffs)
        sigma = tuple(range(d - 1, -1, -1)) if kind == "level" else tuple(rng.permutation(d).tolist())
        L = grid.num_levels(shape)
        for l in range(L - 1):
            G = np.ascontiguousarray(grid.level_grid(x, l))
            cs = grid.decompose_level(G, sigma, kind, degree)
            m_ax = G.shape[axis]
            for rho, c in enumerate(cs):
                sl = grid.region_slices(sigma, rho, d)
                idx = np.indices(G.shape)[axis][sl]
                expect_zero = np.ones(c.shape, dtype=bool)
                ax_rho = sigma[rho]
                if kind == "region" and ax_rho != axis:
                    pass  # interpolation is along another axis of a function constant there
                else:
                    for j in range(1, m_ax, 2):
                        ok = EXACT_DEGREE[grid.stencil_kind(j, m_ax, degree)] >= pdeg
                        expect_zero[idx == j] = ok
                assert np.all(c[expect_zero] == 0.0)
                if pdeg > 0 and (~expect_zero).any():
                    # a non-exact stencil leaves a residual (it can vanish at
                    # isolated points where the error polynomial has a root)
                    assert np.any(c[~expect_zero] != 0.0)


@pytest.mark.parametrize("degree", [1, 3])
@pytest.mark.parametrize("kind", ["level", "region"])
def test_linear_field_on_dyadic_grid_is_all_zero(degree, kind):
    """With every axis of 2^k+1 points no level below the coarsest needs the
    copy stencil, so a linear field has zero coefficients on all of them."""
    x = fieldgen.polynomial_field((17, 17, 17), [[0, 3], [0, -2], [5, 7]])
    L = grid.num_levels(x.shape)
    for l in range(L - 1):
        G = np.ascontiguousarray(grid.level_grid(x, l))
        for c in grid.decompose_level(G, (2, 1, 0), kind, degree):
            assert np.all(c == 0.0)


def _dense_tensor_prediction(G, degree):
    """Per-level prediction of all fine points: kron of 1D matrices applied
    to the coarse values (independent of the oracle's region sweep)."""
    mats = [_prolongation_1d(m, degree) for m in G.shape]
    K = mats[0]
    for Mx in mats[1:]:
        K = np.kron(K, Mx)
    coarse = G[(slice(None, None, 2),) * G.ndim].ravel()
    Kf = K.astype(np.float64)
    return (Kf @ coarse).reshape(G.shape)


@pytest.mark.parametrize("shape", [(8, 8, 8), (9, 9, 9), (6, 9, 7), (10, 5)])
@pytest.mark.parametrize("degree", [1, 3])
def test_per_level_is_tensor_product(shape, degree):
    rng = np.random.default_rng(3)
    G = rng.integers(-50, 50, size=shape).astype(np.float64)
    d = len(shape)
    sigma = tuple(range(d - 1, -1, -1))
    cs = grid.decompose_level(G, sigma, "level", degree)
    pred = _dense_tensor_prediction(G, degree)
    for rho, c in enumerate(cs):
        sl = grid.region_slices(sigma, rho, d)
        np.testing.assert_array_equal(c, G[sl] - pred[sl])


@pytest.mark.parametrize("kind", ["level", "region"])
@pytest.mark.parametrize("degree", [1, 3])
def test_reconstruct_inverts_decompose(kind, degree):
    """With exact coefficients, reconstruction returns the level exactly
    (integer data keeps every float64 operation exact)."""
    rng = np.random.default_rng(4)
    G = rng.integers(-1000, 1000, size=(9, 12, 11)).astype(np.float64)
    sigma = (1, 2, 0) if kind == "region" else (2, 1, 0)
    cs = grid.decompose_level(G, sigma, kind, degree)
    back = grid.reconstruct_level(G[::2, ::2, ::2], G.shape, cs, sigma, kind, degree)
    np.testing.assert_array_equal(back, G)
