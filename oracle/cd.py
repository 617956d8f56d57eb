"""Coefficient decomposition (Section V-B; Algorithm 1 lines on Interleave /
LinearInterpolate / ExtractLevel, and its inverse in Algorithm 2).

The quantized coefficients of one region of the finest level are viewed as a
stack of 2D slices orthogonal to the stacking axis ``a``; each slice is
decomposed by 2D per-level multilinear interpolation with three levels.  The
paper fixes the depth at three (Table II) and uses per-level multilinear
interpolation for its small error propagation.

Integer form (the paper leaves the arithmetic open): with avg(x, y) =
floor((x + y) / 2), for a slice T(u, v) (v the faster of the two remaining
axes; for 2D data the slice is a line and only the v steps exist):

  slice level 1 (from H2, the stride-4 grid):
    v step: points u = 0 mod 4, v = 2 mod 4:  p = avg(T[u, v-2], T[u, v+2])
            (T[u, v-2] if v+2 is outside)
    u step: points u = 2 mod 4, v even:       p = avg(W[u-2, v], W[u+2, v])
            (W[u-2, v] if u+2 is outside), where W is T on H2 and the v-step
            predictions elsewhere (per-level: predictions, not values)
  slice level 0 (from H1, the stride-2 grid, actual values of T):
    v step: points u even, v odd:  p = avg(T[u, v-1], T[u, v+1]) (or copy)
    u step: points u odd:          p = avg(W0[u-1, v], W0[u+1, v]) (or copy)

Outputs: S1 = T on H2, S2 = T - p on H1 \\ H2, S3 = T - p on H0 \\ H1
(R1, R2, R3 of Algorithm 1).  Each output stream lists its points in the
row-major order of the region lattice.  The inverse rebuilds H2, then H1,
then H0, predicting from already rebuilt values; with truncated inputs its
error is at most the sum of the three input errors (a floor average of two
values each off by at most E is off by at most E).
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def _avg(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    return (x + y) >> 1


def _slice_axes(d: int, a: int) -> Tuple[int, ...]:
    """Axis permutation bringing (a, u, v) to the front (3D) or (a, v) (2D)."""
    rest = [ax for ax in range(d) if ax != a]
    return tuple([a] + rest)


def _to_slices(R: np.ndarray, a: int) -> np.ndarray:
    """Region lattice -> (K, Nu, Nv) stack of slices orthogonal to axis a."""
    d = R.ndim
    T = np.transpose(R, _slice_axes(d, a))
    if d == 2:
        T = T[:, None, :]
    return np.ascontiguousarray(T)


def _from_slices(T: np.ndarray, a: int, d: int) -> np.ndarray:
    if d == 2:
        T = T[:, 0, :]
    perm = _slice_axes(d, a)
    inv = np.argsort(perm)
    return np.ascontiguousarray(np.transpose(T, inv))


def class_masks(shape: Tuple[int, ...], a: int) -> List[np.ndarray]:
    """Boolean masks (in lattice axis order) of the S1, S2, S3 points."""
    d = len(shape)
    rest = [ax for ax in range(d) if ax != a]
    if d == 3:
        uax, vax = rest
        shp_u = [1] * d
        shp_u[uax] = shape[uax]
        u = np.arange(shape[uax]).reshape(shp_u)
    else:
        vax = rest[0]
        u = np.zeros([1] * d, dtype=np.int64)
    shp_v = [1] * d
    shp_v[vax] = shape[vax]
    v = np.arange(shape[vax]).reshape(shp_v)
    h2 = (u % 4 == 0) & (v % 4 == 0)
    h1 = (u % 2 == 0) & (v % 2 == 0)
    s1 = np.broadcast_to(h2, shape)
    s2 = np.broadcast_to(h1 & ~h2, shape)
    s3 = np.broadcast_to(~h1, shape)
    return [s1, s2, s3]


def _predict_level1(T: np.ndarray):
    """Predictions on H1 \\ H2 from T on H2 (arrays indexed like T)."""
    K, Nu, Nv = T.shape
    P = np.zeros_like(T)
    W = T.copy()
    for v in range(2, Nv, 4):
        left = T[:, 0::4, v - 2]
        if v + 2 <= Nv - 1:
            p = _avg(left, T[:, 0::4, v + 2])
        else:
            p = left.copy()
        P[:, 0::4, v] = p
        W[:, 0::4, v] = p
    for u in range(2, Nu, 4):
        up = W[:, u - 2, 0::2]
        if u + 2 <= Nu - 1:
            p = _avg(up, W[:, u + 2, 0::2])
        else:
            p = up.copy()
        P[:, u, 0::2] = p
    return P


def _predict_level0(T: np.ndarray):
    """Predictions on H0 \\ H1 from T on H1."""
    K, Nu, Nv = T.shape
    P = np.zeros_like(T)
    W = T.copy()
    for v in range(1, Nv, 2):
        left = T[:, 0::2, v - 1]
        if v + 1 <= Nv - 1:
            p = _avg(left, T[:, 0::2, v + 1])
        else:
            p = left.copy()
        P[:, 0::2, v] = p
        W[:, 0::2, v] = p
    for u in range(1, Nu, 2):
        up = W[:, u - 1, :]
        if u + 1 <= Nu - 1:
            p = _avg(up, W[:, u + 1, :])
        else:
            p = up.copy()
        P[:, u, :] = p
    return P


def _h_masks(Nu: int, Nv: int):
    u = np.arange(Nu)[:, None]
    v = np.arange(Nv)[None, :]
    h2 = (u % 4 == 0) & (v % 4 == 0)
    h1 = (u % 2 == 0) & (v % 2 == 0)
    return h2, h1 & ~h2, ~h1


def forward(R: np.ndarray, a: int) -> List[np.ndarray]:
    """Decompose a region lattice of int64 codes into streams [S1, S2, S3]."""
    R = np.asarray(R, dtype=np.int64)
    d = R.ndim
    assert d in (2, 3)
    T = _to_slices(R, a)
    _, Nu, Nv = T.shape
    m2, m21, m10 = _h_masks(Nu, Nv)
    P1 = _predict_level1(T)
    P0 = _predict_level0(T)
    res = T.copy()
    res[:, m21] = T[:, m21] - P1[:, m21]
    res[:, m10] = T[:, m10] - P0[:, m10]
    Rres = _from_slices(res, a, d)
    return [Rres[m] for m in class_masks(R.shape, a)]


def inverse(streams: List[np.ndarray], shape: Tuple[int, ...], a: int) -> np.ndarray:
    """Recompose a region lattice from (possibly truncated) streams [S1, S2, S3]."""
    d = len(shape)
    Rres = np.zeros(shape, dtype=np.int64)
    for m, s in zip(class_masks(shape, a), streams):
        Rres[m] = s
    res = _to_slices(Rres, a)
    _, Nu, Nv = res.shape
    m2, m21, m10 = _h_masks(Nu, Nv)
    T = np.zeros_like(res)
    T[:, m2] = res[:, m2]
    P1 = _predict_level1(T)
    T[:, m21] = res[:, m21] + P1[:, m21]
    P0 = _predict_level0(T)
    T[:, m10] = res[:, m10] + P0[:, m10]
    return _from_slices(T, a, d)
