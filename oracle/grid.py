"""Multilevel grids, 1D interpolation stencils and per-level / per-region
decomposition and reconstruction of one level (Section IV; Algorithms 1 and 2).

Conventions
-----------
* Arrays are row-major; the last axis is the fastest-varying one ("x").
* Level l keeps the points whose index on every axis is a multiple of 2**l
  (Section IV: each level halves the resolution of the previous one).  The
  points of level l, taken on their own, form the *compact grid* G_l; on an
  axis of length n it has (n - 1) // 2**l + 1 points.  On G_l the points of
  level l + 1 are the even compact indices and the points interpolated at
  level l are the others.
* Region rho of a level (rho = 0..d-1, in pass order sigma) holds the points
  that are odd on axis sigma[rho], even on the axes sigma[j] with j > rho and
  anything on the axes sigma[j] with j < rho (Section IV: the points
  interpolated along one dimension form a region; Section VI-C: per-level
  interpolation is the same as interpolating the regions one after the other
  along x, then y, then z).  A region, read in row-major order of its own
  index ranges, is its *lattice*.

Stencils (cubic with quadratic/linear fall-backs near the ends of an axis)
--------------------------------------------------------------------------
For an odd compact index j on an axis of compact length m, with
a = v[j-3], b = v[j-1], c = v[j+1], e = v[j+3]:

  copy      j+1 > m-1                      p = b
  cubic     j-3 >= 0 and j+3 <= m-1         p = (9*(b+c) - (a+e)) / 16
  lquad     j-3 <  0 and j+3 <= m-1         p = (3*b + 6*c - e) / 8
  rquad     j-3 >= 0 and j+3 >  m-1         p = (6*b + 3*c - a) / 8
  linear    otherwise (or degree 1)         p = (b + c) / 2

The cubic weights are the 4-point interpolating cubic; the quadratic ones are
the Lagrange weights through the three available neighbours.  Every weight is
dyadic.  The float64 expressions below fix the operation order exactly; the
GPU evaluates the same expressions without contraction.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def num_levels(shape: Sequence[int]) -> int:
    """Default L: 1 + ceil(log2(max n - 1)), so the coarsest level has 1-2 points per axis."""
    nmax = max(int(s) for s in shape)
    if nmax <= 2:
        return 1
    return 1 + (nmax - 2).bit_length()


def compact_len(n: int, level: int) -> int:
    return (int(n) - 1) // (1 << level) + 1


def level_grid(x: np.ndarray, level: int) -> np.ndarray:
    """Values of level ``level`` as a compact grid (a strided view)."""
    s = 1 << level
    return x[(slice(None, None, s),) * x.ndim]


def stencil_kind(j: int, m: int, degree: int) -> str:
    if j + 1 > m - 1:
        return "copy"
    if degree == 1:
        return "linear"
    left = j - 3 >= 0
    right = j + 3 <= m - 1
    if left and right:
        return "cubic"
    if right:
        return "lquad"
    if left:
        return "rquad"
    return "linear"


def stencil_apply(kind: str, a, b, c, e):
    if kind == "cubic":
        t1 = b + c
        t2 = a + e
        return (9.0 * t1 - t2) * 0.0625
    if kind == "lquad":
        return ((3.0 * b + 6.0 * c) - e) * 0.125
    if kind == "rquad":
        return ((6.0 * b + 3.0 * c) - a) * 0.125
    if kind == "linear":
        return (b + c) * 0.5
    return b * 1.0


def region_slices(sigma: Sequence[int], rho: int, d: int) -> Tuple[slice, ...]:
    sl: List[slice] = [slice(None)] * d
    for j, ax in enumerate(sigma):
        if j < rho:
            sl[ax] = slice(None)
        elif j == rho:
            sl[ax] = slice(1, None, 2)
        else:
            sl[ax] = slice(0, None, 2)
    return tuple(sl)


def region_shape(shape_m: Sequence[int], sigma: Sequence[int], rho: int) -> Tuple[int, ...]:
    d = len(shape_m)
    out = [0] * d
    for j, ax in enumerate(sigma):
        m = int(shape_m[ax])
        if j < rho:
            out[ax] = m
        elif j == rho:
            out[ax] = m // 2
        else:
            out[ax] = (m + 1) // 2
    return tuple(out)


def predict_region(V: np.ndarray, sigma: Sequence[int], rho: int, degree: int) -> np.ndarray:
    """Predictions for every point of region ``rho`` by the 1D stencil along
    axis sigma[rho], reading its neighbours from ``V`` (float64 compact grid)."""
    d = V.ndim
    ax = sigma[rho]
    m = V.shape[ax]
    sl = list(region_slices(sigma, rho, d))
    P = np.empty(region_shape(V.shape, sigma, rho), dtype=np.float64)
    for t, j in enumerate(range(1, m, 2)):
        kind = stencil_kind(j, m, degree)

        def tap(o: int):
            if j + o < 0 or j + o > m - 1:
                return None
            s = list(sl)
            s[ax] = j + o
            return V[tuple(s)]

        p = stencil_apply(kind, tap(-3), tap(-1), tap(1), tap(3))
        idx = [slice(None)] * d
        idx[ax] = t
        P[tuple(idx)] = p
    return P


def decompose_level(G: np.ndarray, sigma: Sequence[int], kind: str, degree: int) -> List[np.ndarray]:
    """Coefficients (original minus prediction) of one level, region by region.

    ``G`` is the float64 compact grid of this level's points (original data).
    Per-level (Section IV): each prediction uses only the level above, i.e.
    the predictions of earlier regions stand in for their points, which makes
    the result the tensor-product interpolation of the level above.
    Per-region (Section IV): each pass reads the original values of the
    points already processed; no pre-quantization is applied.
    Returns one float64 array per region, in lattice shape.
    """
    d = G.ndim
    V = G.copy()
    out = []
    for rho in range(d):
        sl = region_slices(sigma, rho, d)
        src = V if kind == "level" else G
        P = predict_region(src, sigma, rho, degree)
        out.append(G[sl] - P)
        if kind == "level":
            V[sl] = P
    return out


def reconstruct_level(coarse: np.ndarray, shape_m: Sequence[int], dq: List[np.ndarray],
                      sigma: Sequence[int], kind: str, degree: int) -> np.ndarray:
    """Inverse of ``decompose_level`` (Algorithm 2): values of this level from
    the reconstructed level above (``coarse``) and the dequantized
    coefficients ``dq`` (one float64 lattice per region).

    Per-level: all predictions come from the level above; each point is then
    prediction + coefficient.  Per-region: pass rho reads the values already
    reconstructed by earlier passes, so errors travel across regions.
    """
    d = len(shape_m)
    V = np.zeros(tuple(int(s) for s in shape_m), dtype=np.float64)
    V[(slice(None, None, 2),) * d] = coarse
    out = V.copy() if kind == "level" else None
    for rho in range(d):
        sl = region_slices(sigma, rho, d)
        P = predict_region(V, sigma, rho, degree)
        if kind == "level":
            V[sl] = P
            out[sl] = P + dq[rho]
        else:
            V[sl] = P + dq[rho]
    return out if kind == "level" else V
