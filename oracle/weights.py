"""Error-propagation weights of the multilevel interpolation (Section V-C
bitplane-to-error mapping; the paper cites the estimators of its baselines but
gives no formula).

Reconstruction is linear in the coefficients.  Along one axis, an error on the
points of level l reaches the full grid through the chain of 1D prolongations
s_0 o s_1 o ... o s_(l-1), where s_j keeps the points of level j+1 and fills
the others with the stencil of ``oracle.grid`` (the identity if the axis has
no points to fill at level j).  Interpolation of a level is the tensor product
of these 1D maps, so the max-row-abs-sum (infinity norm) and max-column-abs-sum
(1-norm) of the multi-dimensional map are products of the per-axis ones.

  lam_inf[a][l], lam_1[a][l]   norms of the axis-a chain from level l,
                               computed exactly in integers (every weight is
                               a multiple of 1/16) and rounded once to float64.

Group weights (axis order a = 0..d-1, multiplied left to right):
  per-level level l / coarsest:  every axis at level l (L-1 for the coarsest)
  per-region (l, rho):           axes sigma[j], j <= rho at level l; axes
                                 sigma[j], j > rho at level l+1 (the level-l
                                 passes along those axes carry the error on)
  w_g   = prod_a lam_inf[a][lev_a]                       (max-error weight)
  rho_g = sqrt(n_g / n) * prod_a sqrt(lam_inf * lam_1)   (RMSE weight, from
          ||P e||_2 <= sqrt(||P||_1 ||P||_inf) ||e||_2 and ||e||_2 <= sqrt(n_g) max|e|)
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import List, Sequence, Tuple

import numpy as np

from .grid import compact_len, stencil_kind

_LIMIT = 1 << 60


def _prolong_columns(P: np.ndarray, m_fine: int, degree: int) -> np.ndarray:
    """Right-multiply P (n x m_fine, values on the finer level j) by the
    prolongation s_j (m_fine x m_coarse), scaled by 16."""
    n = P.shape[0]
    m_coarse = (m_fine + 1) // 2
    out = np.zeros((n, m_coarse), dtype=np.int64)
    for k in range(m_coarse):
        out[:, k] += 16 * P[:, 2 * k]
    for i in range(1, m_fine, 2):
        kind = stencil_kind(i, m_fine, degree)
        if kind == "cubic":
            terms = [((i - 3) // 2, -1), ((i - 1) // 2, 9), ((i + 1) // 2, 9), ((i + 3) // 2, -1)]
        elif kind == "lquad":
            terms = [((i - 1) // 2, 6), ((i + 1) // 2, 12), ((i + 3) // 2, -2)]
        elif kind == "rquad":
            terms = [((i - 3) // 2, -2), ((i - 1) // 2, 12), ((i + 1) // 2, 6)]
        elif kind == "linear":
            terms = [((i - 1) // 2, 8), ((i + 1) // 2, 8)]
        else:
            terms = [((i - 1) // 2, 16)]
        for k, wgt in terms:
            out[:, k] += wgt * P[:, i]
    assert np.abs(out).max(initial=0) < _LIMIT
    return out


def axis_norms(n: int, L: int, degree: int) -> Tuple[List[float], List[float]]:
    """(lam_inf[l], lam_1[l]) for l = 0..L-1 on an axis of length n."""
    lam_inf, lam_1 = [1.0], [1.0]
    P = np.eye(n, dtype=np.int64)
    for l in range(1, L):
        P = _prolong_columns(P, compact_len(n, l - 1), degree)
        den = 16 ** l
        rows = np.abs(P).sum(axis=1)
        cols = np.abs(P).sum(axis=0)
        assert rows.max() < _LIMIT and cols.max() < _LIMIT
        lam_inf.append(float(Fraction(int(rows.max()), den)))
        lam_1.append(float(Fraction(int(cols.max()), den)))
    return lam_inf, lam_1


def all_axis_norms(shape: Sequence[int], L: int, degree: int):
    return [axis_norms(int(n), L, degree) for n in shape]


def group_weights(norms, levs: Sequence[int], n_g: int, n: int) -> Tuple[float, float]:
    """(w_g, rho_g) for a group whose axis a sits at level levs[a]."""
    w = 1.0
    r = math.sqrt(n_g / n)
    for a, l in enumerate(levs):
        li, l1 = norms[a][0][l], norms[a][1][l]
        w = w * li
        r = r * math.sqrt(li * l1)
    return w, r


def region_levels(sigma: Sequence[int], rho: int, level: int, d: int) -> List[int]:
    levs = [0] * d
    for j, ax in enumerate(sigma):
        levs[ax] = level if j <= rho else level + 1
    return levs
