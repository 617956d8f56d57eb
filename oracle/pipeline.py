"""Refactoring (Algorithm 1), retrieval (Algorithm 2) and target-driven
pipeline selection (Section VI-A), oracle side.

Refactoring
  1. range pass: min, max, max|x|; non-finite input is rejected
  2. every level l < L-1 is decomposed on its compact grid (Section IV); the
     coarsest level keeps its values as coefficients
  3. error-bounded quantization per group (Section V-C keeps the largest
     coefficient of a level as metadata): M_g = max|c|, (m, E_g) = frexp(M_g),
     Delta_g = 2^(E_g - P), q = rint(c * 2^(P - E_g)), so |c - Delta_g q| <=
     Delta_g / 2 and |q| <= 2^P; P = 29 for float32 input, 52 for float64.
     Groups: per-level, one per level; per-region, one per (level, region);
     plus the coarsest level.  A group whose coefficients are all zero has
     Delta_g = 0.
  4. coefficient decomposition of every region of level 0 when enabled
     (Section V-B, ``oracle.cd``)
  5. generic bitplane encoding of every stream (``oracle.bitplane``)

Streams, in unit order: the coarsest level (row-major); then for
l = L-2 .. 0 either the level (per-level: its regions' lattices one after the
other) or one stream per region (per-region); under decomposition each
region of level 0 gives S1, S2, S3 instead.

Retrieval decodes the planned planes, undoes the decomposition, and
reconstructs from the coarsest level down (Algorithm 2), in float64, casting
once to the input type.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import bitplane, cd, grid, weights
from .plan import BelowFloor, Plan, Unit, build_staircase, eps_fp, greedy_sequence, make_plan, plan_bytes
from .scheme import Scheme, Target


class NonFinite(ValueError):
    pass


@dataclass
class Group:
    key: tuple
    n: int
    M: float
    E: int
    delta: float
    w: float
    rho: float
    cd: str = "none"            # "none", "sum" (per-region CD), "stair" (per-level CD)
    wd_inf: float = 0.0
    wd_2: float = 0.0


@dataclass
class Stream:
    key: tuple
    group: int
    meta: bitplane.StreamMeta
    blob: bytes
    codes: np.ndarray


@dataclass
class Refactored:
    shape: Tuple[int, ...]
    dtype: np.dtype
    scheme: Scheme
    L: int
    P: int
    xmin: float
    xmax: float
    A: float
    sigma: Tuple[int, ...]
    groups: List[Group] = field(default_factory=list)
    streams: List[Stream] = field(default_factory=list)
    units: List[Unit] = field(default_factory=list)
    group_units: Dict[int, List[int]] = field(default_factory=dict)
    group_order: List[int] = field(default_factory=list)
    lattices: Dict[Tuple[int, int], Tuple[int, ...]] = field(default_factory=dict)
    eps_fp: float = 0.0
    meta_bytes: int = 0
    _seq: Dict[str, tuple] = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))

    @property
    def range(self) -> float:
        return self.xmax - self.xmin

    def sequence(self, mode: str):
        if mode not in self._seq:
            self._seq[mode] = greedy_sequence(self, mode)
        return self._seq[mode]


def _precision(dtype) -> int:
    dt = np.dtype(dtype)
    if dt == np.float32:
        return 29
    if dt == np.float64:
        return 52
    raise TypeError(f"unsupported dtype {dt}")


def quantize(c: np.ndarray, M: float, P: int):
    """Exponent-aligned quantization of one group (returns E, Delta, int64 codes)."""
    if not (M > 0.0):
        return 0, 0.0, np.zeros(c.shape, dtype=np.int64)
    _, E = math.frexp(M)
    q = np.rint(np.ldexp(c, P - E)).astype(np.int64)
    return E, math.ldexp(1.0, E - P), q


def refactor(x: np.ndarray, scheme: Scheme = Scheme(), precision: Optional[int] = None) -> Refactored:
    """``precision`` overrides P (tests use a small P to enumerate plans)."""
    x = np.asarray(x)
    P = _precision(x.dtype) if precision is None else int(precision)
    d = x.ndim
    assert 1 <= d <= 3
    shape = tuple(int(s) for s in x.shape)
    xf = x.astype(np.float64)
    if not np.all(np.isfinite(xf)):
        raise NonFinite("input holds NaN or Inf")
    if scheme.cd_axis is not None:
        assert d >= 2 and 0 <= scheme.cd_axis < d, "decomposition needs 2D/3D data"
    L = scheme.levels or grid.num_levels(shape)
    sigma = scheme.pass_order(d)
    ref = Refactored(shape=shape, dtype=x.dtype, scheme=scheme, L=L, P=P,
                     xmin=float(xf.min()), xmax=float(xf.max()),
                     A=float(np.abs(xf).max()), sigma=sigma)
    n = xf.size
    norms = weights.all_axis_norms(shape, L, scheme.degree)

    # Decomposition, level by level (levels are independent: each reads only
    # the original values of its own points).
    coeffs: Dict[Tuple[int, int], np.ndarray] = {}
    for l in range(L - 1):
        G = np.ascontiguousarray(grid.level_grid(xf, l))
        for rho, c in enumerate(grid.decompose_level(G, sigma, scheme.kind, scheme.degree)):
            coeffs[(l, rho)] = c
            ref.lattices[(l, rho)] = c.shape
    coarse = np.ascontiguousarray(grid.level_grid(xf, L - 1))
    ref.lattices[("c",)] = coarse.shape

    def add_group(key, c_list, levs, cd_kind="none"):
        vals = np.concatenate([c.ravel() for c in c_list]) if c_list else np.zeros(0)
        M = float(np.abs(vals).max()) if vals.size else 0.0
        E, delta, q = quantize(vals, M, P)
        w, r = weights.group_weights(norms, levs, vals.size, n)
        grp = Group(key=key, n=int(vals.size), M=M, E=E, delta=delta, w=w, rho=r, cd=cd_kind)
        grp.wd_inf = w * delta
        grp.wd_2 = r * delta
        ref.groups.append(grp)
        return len(ref.groups) - 1, q

    def add_stream(key, g, codes):
        if scheme.encoding == "generic":
            blob, meta = bitplane.encode(codes, lossless=scheme.lossless)
        else:
            blob, meta = bitplane.encode_nb(codes, xor=scheme.encoding == "negabinary_xor", lossless=scheme.lossless)
        ref.streams.append(Stream(key=key, group=g, meta=meta, blob=blob, codes=np.asarray(codes, np.int64).ravel()))
        return len(ref.streams) - 1

    def add_cd(level, rho, g, q_lattice, region_streams):
        trip = []
        for t, s in enumerate(cd.forward(q_lattice, scheme.cd_axis)):
            trip.append(add_stream(("cd", level, rho, t + 1), g, s))
        region_streams.append(trip)
        return trip

    units: List[Unit] = []

    g, q = add_group(("c",), [coarse], [L - 1] * d)
    s = add_stream(("c",), g, q)
    units.append(Unit(group=g, kind="plane", stream=s, meta=ref.streams[s].meta))

    for l in range(L - 2, -1, -1):
        use_cd = scheme.cd_axis is not None and l == 0
        if scheme.kind == "level":
            cl = [coeffs[(l, rho)] for rho in range(d)]
            g, q = add_group(("l", l), cl, [l] * d, "stair" if use_cd else "none")
            if not use_cd:
                s = add_stream(("l", l), g, q)
                units.append(Unit(group=g, kind="plane", stream=s, meta=ref.streams[s].meta))
            else:
                region_streams: List[List[int]] = []
                off = 0
                for rho in range(d):
                    shp = cl[rho].shape
                    cnt = int(np.prod(shp))
                    add_cd(l, rho, g, q[off:off + cnt].reshape(shp), region_streams)
                    off += cnt
                units.append(build_staircase(g, region_streams, [st.meta for st in ref.streams]))
        else:
            for rho in range(d):
                c = coeffs[(l, rho)]
                levs = weights.region_levels(sigma, rho, l, d)
                g, q = add_group(("r", l, rho), [c], levs, "sum" if use_cd else "none")
                if not use_cd:
                    s = add_stream(("r", l, rho), g, q)
                    units.append(Unit(group=g, kind="plane", stream=s, meta=ref.streams[s].meta))
                else:
                    trip = add_cd(l, rho, g, q.reshape(c.shape), [])
                    for s in trip:
                        units.append(Unit(group=g, kind="plane", stream=s, meta=ref.streams[s].meta))

    ref.units = units
    for u, unit in enumerate(units):
        ref.group_units.setdefault(unit.group, []).append(u)
        if unit.group not in ref.group_order:
            ref.group_order.append(unit.group)
    ref.eps_fp = eps_fp(ref)
    nseg = sum(len(u.seg_bytes) for u in units if u.kind == "stair")
    # with the lossless stage every plane also records its nonzero word count
    per_plane = 8 if scheme.lossless else 4
    ref.meta_bytes = (64 + 16 * len(ref.groups) + 16 * len(ref.streams)
                      + per_plane * sum(st.meta.B for st in ref.streams) + 8 * nseg)
    return ref


def target_tau(ref: Refactored, target: Target):
    """(tau, mode) for a target: mode "inf" bounds max error, "l2" bounds RMSE."""
    if target.kind == "abs":
        return float(target.value), "inf"
    if target.kind == "rel":
        return float(target.value) * ref.range, "inf"
    if target.kind == "rmse":
        return float(target.value), "l2"
    if target.kind == "psnr":
        return ref.range * 10.0 ** (-float(target.value) / 20.0), "l2"
    raise ValueError(target.kind)


def plan(ref: Refactored, target: Target) -> Plan:
    tau, mode = target_tau(ref, target)
    return make_plan(ref, tau, mode)


def decode_codes(ref: Refactored, k: List[int]) -> List[np.ndarray]:
    return [bitplane.decode(st.blob, st.meta, k[s]) for s, st in enumerate(ref.streams)]


def retrieve(ref: Refactored, pl, codes: Optional[List[np.ndarray]] = None) -> np.ndarray:
    """Reconstruct the field from the planes of plan ``pl`` (a Plan or a
    per-stream plane list)."""
    k = pl.planes if isinstance(pl, Plan) else list(pl)
    if codes is None:
        codes = decode_codes(ref, k)
    d = len(ref.shape)
    sc = ref.scheme
    by_key = {st.key: i for i, st in enumerate(ref.streams)}
    gc = ref.groups[ref.streams[by_key[("c",)]].group]
    x = codes[by_key[("c",)]].astype(np.float64).reshape(ref.lattices[("c",)]) * gc.delta
    for l in range(ref.L - 2, -1, -1):
        shape_m = tuple(grid.compact_len(nn, l) for nn in ref.shape)
        use_cd = sc.cd_axis is not None and l == 0
        dq = []
        if sc.kind == "level" and not use_cd:
            s = by_key[("l", l)]
            delta = ref.groups[ref.streams[s].group].delta
            off = 0
            for rho in range(d):
                shp = ref.lattices[(l, rho)]
                cnt = int(np.prod(shp))
                dq.append(codes[s][off:off + cnt].astype(np.float64).reshape(shp) * delta)
                off += cnt
        else:
            for rho in range(d):
                shp = ref.lattices[(l, rho)]
                if use_cd:
                    trip = [by_key[("cd", l, rho, t)] for t in (1, 2, 3)]
                    qr = cd.inverse([codes[s] for s in trip], shp, sc.cd_axis)
                    delta = ref.groups[ref.streams[trip[0]].group].delta
                else:
                    s = by_key[("r", l, rho)]
                    qr = codes[s].reshape(shp)
                    delta = ref.groups[ref.streams[s].group].delta
                dq.append(qr.astype(np.float64) * delta)
        x = grid.reconstruct_level(x, shape_m, dq, ref.sigma, sc.kind, sc.degree)
    return x.astype(ref.dtype)


def quantized_field(ref: Refactored) -> np.ndarray:
    """X_q: the reconstruction from every plane."""
    return retrieve(ref, [st.meta.B for st in ref.streams])


# --------------------------------------------------------------------------
# Target-driven pipeline selection (Section VI-A, Table I).
# --------------------------------------------------------------------------

TUNING_TOLERANCES = (1e-3, 5e-4, 1e-4, 5e-5, 1e-5, 5e-6, 1e-6, 5e-7, 1e-7)


def sample_blocks(x: np.ndarray, block: Optional[int] = None, every: Optional[int] = None):
    """Regular sample of the field: blocks of side ``block`` at every
    ``every``-th block position along each axis (about 1% of a 3D field with
    32^3 blocks every 5th position; 128^2 blocks every 10th position in 2D).
    At least one block is taken."""
    d = x.ndim
    if block is None:
        block = {1: 4096, 2: 128, 3: 32}[d]
    if every is None:
        every = {1: 100, 2: 10, 3: 5}[d]
    out = []
    ranges = []
    for a in range(d):
        nb = max(1, x.shape[a] // block)
        ranges.append(range(0, nb, every))
    for pos in itertools.product(*ranges):
        sl = tuple(slice(p * block, min(x.shape[a], (p + 1) * block)) for a, p in enumerate(pos))
        out.append(np.ascontiguousarray(x[sl]))
    return out


def candidates(d: int, mode: str):
    """Interpolation candidates (cd off): per-level (error-bound mode only)
    and per-region with every dimension order in lexicographic order."""
    c = []
    if mode == "eb":
        c.append(Scheme(kind="level"))
    for perm in itertools.permutations(range(d)):
        c.append(Scheme(kind="region", order=tuple(perm)))
    return c


def _sample_bytes(blocks, scheme: Scheme, tol: float, rng: float, mode: str) -> int:
    """Plan bytes summed over the sample blocks; a block whose floor is above
    the tolerance counts every plane it has."""
    total = 0
    for blk in blocks:
        ref = refactor(blk, scheme)
        try:
            total += make_plan(ref, tol * rng, "inf" if mode == "eb" else "l2").bytes
        except BelowFloor:
            total += plan_bytes(ref, [st.meta.B for st in ref.streams])
    return total


def _vote(blocks, cands, rng, mode):
    votes = [0] * len(cands)
    for tol in TUNING_TOLERANCES:
        sizes = [_sample_bytes(blocks, c, tol, rng, mode) for c in cands]
        best = min(range(len(cands)), key=lambda i: (sizes[i], i))
        votes[best] += 1
    return max(range(len(cands)), key=lambda i: (votes[i], -i))


def select_pipeline(x: np.ndarray, mode: str = "eb") -> Scheme:
    """Vote over the tuning tolerances on a ~1% sample (Section VI-A).

    Interpolation is chosen first with decomposition off; decomposition
    (none, then axes 0..d-1) is then chosen for the winning interpolation.
    In PSNR mode a tolerance means an RMSE of tol * range.
    """
    x = np.asarray(x)
    d = x.ndim
    xf = x.astype(np.float64)
    rng = float(xf.max()) - float(xf.min())
    blocks = sample_blocks(x)
    cands = candidates(d, mode)
    best = cands[_vote(blocks, cands, rng, mode)]
    if d >= 2:
        cd_cands = [best] + [Scheme(kind=best.kind, degree=best.degree, order=best.order, cd_axis=a)
                             for a in range(d)]
        best = cd_cands[_vote(blocks, cd_cands, rng, mode)]
    return best
