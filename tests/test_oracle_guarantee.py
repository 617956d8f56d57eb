"""Pins of the error model (Section V-C) and the retrieval guarantee
(Section III-A): brute-force operator norms, the closed form of linear
weights, the max-error bound on every greedy plan and on random plans, the
PSNR target, nesting and minimality of plans."""
import itertools
import math

import numpy as np
import pytest

import fieldgen
import oracle
from oracle import Scheme, Target, grid, weights
from oracle.plan import BelowFloor, bound_for_planes
from oracle.pipeline import quantized_field, refactor, retrieve


SCHEMES = [Scheme("level"), Scheme("region"), Scheme("level", cd_axis=0), Scheme("region", cd_axis=1, order=(0, 2, 1)),
           Scheme("level", degree=1), Scheme("region", degree=1, order=(1, 0, 2), cd_axis=2)]


def _impulse_matrix(shape, kind, degree, sigma, group_key):
    """Dense map from a group's coefficients (Delta = 1) to the full grid,
    built by reconstructing unit impulses one at a time."""
    d = len(shape)
    L = grid.num_levels(shape)
    lat = {}
    for l in range(L - 1):
        shp = tuple(grid.compact_len(n, l) for n in shape)
        for rho in range(d):
            lat[(l, rho)] = grid.region_shape(shp, sigma, rho)
    coarse_shape = tuple(grid.compact_len(n, L - 1) for n in shape)

    def recon(coarse, dqs):
        x = coarse
        for l in range(L - 2, -1, -1):
            shp = tuple(grid.compact_len(n, l) for n in shape)
            x = grid.reconstruct_level(x, shp, [dqs[(l, r)] for r in range(d)], sigma, kind, degree)
        return x.ravel()

    def zeros():
        return np.zeros(coarse_shape), {k: np.zeros(v) for k, v in lat.items()}

    cols = []
    if group_key[0] == "c":
        for i in range(int(np.prod(coarse_shape))):
            c0, dq = zeros()
            c0.ravel()[i] = 1.0
            cols.append(recon(c0, dq))
    else:
        keys = [(group_key[1], r) for r in range(d)] if group_key[0] == "l" else [(group_key[1], group_key[2])]
        for key in keys:
            for i in range(int(np.prod(lat[key]))):
                c0, dq = zeros()
                dq[key].ravel()[i] = 1.0
                cols.append(recon(c0, dq))
    return np.stack(cols, axis=1) if cols else np.zeros((int(np.prod(shape)), 0))


@pytest.mark.parametrize("shape", [(8, 8, 8), (9, 9, 9), (6, 11), (13,)])
@pytest.mark.parametrize("kind", ["level", "region"])
@pytest.mark.parametrize("degree", [1, 3])
def test_weights_bound_brute_force_norms(shape, kind, degree):
    d = len(shape)
    x = np.zeros(shape)
    sc = Scheme(kind, degree=degree, order=tuple(range(d))[::-1] if kind == "level" else tuple(np.roll(np.arange(d), 1)))
    ref = refactor(x, sc)
    n = x.size
    for g in ref.groups:
        Pm = _impulse_matrix(shape, kind, degree, ref.sigma, g.key)
        if Pm.shape[1] == 0:
            continue
        row_inf = np.abs(Pm).sum(axis=1).max()
        col_1 = np.abs(Pm).sum(axis=0).max()
        assert row_inf <= g.w * (1 + 1e-12), (g.key, row_inf, g.w)
        l2 = np.linalg.norm(Pm, 2)
        # rho_g bounds ||P||_2 * sqrt(n_g / n)
        assert l2 * math.sqrt(g.n / n) <= g.rho * (1 + 1e-12) + 1e-15
        if g.key[0] == "c":
            # the coarsest group spans a whole tensor-product grid: attained
            assert row_inf == pytest.approx(g.w, rel=1e-12)
        if degree == 1:
            assert g.w == 1.0
        assert col_1 > 0


def test_linear_weights_are_one():
    for n in (5, 17, 100, 513):
        li, l1 = weights.axis_norms(n, grid.num_levels((n,)), 1)
        assert li == [1.0] * len(li)


def test_cubic_weights_stay_small():
    li, _ = weights.axis_norms(512, 10, 3)
    assert max(li) < 1.26 and li[0] == 1.0


@pytest.mark.parametrize("sc", SCHEMES, ids=str)
def test_eb_ladder_guarantee(config1_field, sc):
    ref = refactor(config1_field, sc)
    x = config1_field.astype(np.float64)
    prev = None
    for rel in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7):
        tau = rel * ref.range
        try:
            pl = oracle.plan(ref, Target("rel", rel))
        except BelowFloor:
            assert bound_for_planes(ref, [st.meta.B for st in ref.streams], "inf") > tau
            continue
        xr = retrieve(ref, pl).astype(np.float64)
        assert np.abs(xr - x).max() <= tau
        assert pl.bound <= tau
        assert bound_for_planes(ref, pl.planes, "inf") == pytest.approx(pl.bound, rel=0, abs=0)
        if prev is not None:                      # nesting
            assert all(a >= b for a, b in zip(pl.planes, prev.planes))
        if pl.nsteps > 0:                          # minimality of the greedy prefix
            E0, seq = ref.sequence("inf")
            before = seq[pl.nsteps - 2][2] if pl.nsteps >= 2 else E0
            assert before > tau
        prev = pl


@pytest.mark.parametrize("sc", SCHEMES[:4], ids=str)
def test_psnr_guarantee(config1_field, sc):
    ref = refactor(config1_field, sc)
    x = config1_field.astype(np.float64)
    for psnr in (40, 60, 80, 100):
        pl = oracle.plan(ref, Target("psnr", psnr))
        xr = retrieve(ref, pl).astype(np.float64)
        rmse = math.sqrt(np.mean((xr - x) ** 2))
        assert rmse <= ref.range * 10 ** (-psnr / 20)
        assert 20 * math.log10(ref.range / rmse) >= psnr


@pytest.mark.parametrize("sc", SCHEMES, ids=str)
def test_full_retrieval_is_quantized_field(config1_field, sc):
    ref = refactor(config1_field, sc)
    xq = quantized_field(ref)
    x = config1_field.astype(np.float64)
    full = bound_for_planes(ref, [st.meta.B for st in ref.streams], "inf")
    assert np.abs(xq.astype(np.float64) - x).max() <= full
    # codes decode to themselves
    for st in ref.streams:
        np.testing.assert_array_equal(oracle.bitplane.decode(st.blob, st.meta, st.meta.B), st.codes)


@pytest.mark.parametrize("sc", [Scheme("level"), Scheme("region", order=(0, 1, 2)), Scheme("level", cd_axis=0),
                                Scheme("region", cd_axis=2)], ids=str)
def test_random_plans_respect_bound_small_precision(sc):
    """With P = 6 the 8^3 field has few planes per stream; random plane
    vectors (not only greedy ones) must respect the model bound."""
    x = fieldgen.gaussian_bumps((8, 8, 8), seed=5, nbumps=3, dtype=np.float64)
    ref = refactor(x, sc, precision=6)
    rng = np.random.default_rng(0)
    Bs = [st.meta.B for st in ref.streams]
    trials = list(itertools.islice(itertools.product(*[range(b + 1) for b in Bs]), 0, 50))
    trials += [[int(rng.integers(0, b + 1)) for b in Bs] for _ in range(300)]
    for k in trials:
        xr = retrieve(ref, list(k)).astype(np.float64)
        assert np.abs(xr - x).max() <= bound_for_planes(ref, list(k), "inf")
        rmse = math.sqrt(np.mean((xr - x) ** 2))
        assert rmse <= bound_for_planes(ref, list(k), "l2")


def test_constant_field_relative_target_is_below_floor():
    x = np.full((9, 9, 9), 3.0, dtype=np.float32)
    ref = refactor(x, Scheme("level"))
    with pytest.raises(BelowFloor):
        oracle.plan(ref, Target("rel", 1e-3))
    pl = oracle.plan(ref, Target("abs", 1e-3))
    np.testing.assert_array_equal(retrieve(ref, pl), x)


@pytest.mark.parametrize("shape", [(1,), (2,), (3, 1), (1, 1, 1), (2, 3, 5), (17,), (33, 5)])
def test_tiny_and_degenerate_shapes(shape):
    x = fieldgen.polynomial_field(shape, [[1, 2, 0, 1]] * len(shape)).astype(np.float32) / 7
    for sc in (Scheme("level"), Scheme("region")):
        ref = refactor(x, sc)
        xq = quantized_field(ref)
        assert np.abs(xq.astype(np.float64) - x).max() <= bound_for_planes(ref, [s.meta.B for s in ref.streams], "inf")


def test_nonfinite_rejected():
    x = np.zeros((4, 4, 4), dtype=np.float32)
    x[1, 2, 3] = np.nan
    with pytest.raises(oracle.pipeline.NonFinite):
        refactor(x)


def test_float64_input(config1_field):
    x = config1_field.astype(np.float64)
    ref = refactor(x, Scheme("level", cd_axis=0))
    assert ref.P == 52
    for rel in (1e-3, 1e-7, 1e-10):
        pl = oracle.plan(ref, Target("rel", rel))
        xr = retrieve(ref, pl)
        assert np.abs(xr - x).max() <= rel * ref.range
