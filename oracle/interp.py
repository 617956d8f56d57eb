"""The paper's retrieval interpreters (Section V-C; Algorithm 2
"RetrievalInterpreter"), oracle side: dynamic programming for per-region
interpolation and best-first search with pruning and incremental invocation
for per-level interpolation with coefficient decomposition.  The paper names
both (the dynamic program is the one of its reference on progressive
interpolation compressors) but gives neither; the readings below are this
project's.

The planning problem.  A plan takes k_u steps of every unit u (planes of a
stream, or segments of the level-0 staircase).  The error model of
``oracle.plan`` is a sum over groups, and within a group the error is one
unit's, the sum of its units' (per-region decomposition) or the staircase's
ceiling, so it is additive over units:

  E(k) = sum_g wd_g * (0.5 + e_g(k)) + eps_fp,   e_g = sum_{u in g} e_u(k_u)

The interpreters minimise the bytes a retrieval must fetch, sum_u c_u(k_u),
subject to E(k) <= tau.  Incremental invocation: planes already resident
(fetched by earlier retrievals of the same handle) cost nothing, so c_u counts
only planes beyond them and k_u never goes below the resident steps.  Both
interpreters return the greedy plan (``oracle.plan``) when it fetches no more
bytes than what they find, so they are never worse than it.

Dynamic programming (per-region interpolation).  The error budget
R = tau - eps_fp - sum_g 0.5 wd_g is split into D = 2048 equal parts q; each
unit's error term a_u(k) = wd_g * e_u(k) is rounded up to a whole number of
parts, A_u(k) = ceil(a_u(k) / q), and a table over units and part counts
keeps, for every count b, the fewest bytes whose parts sum to at most b
(ties to the smaller step count).  Rounding up keeps every plan within the
budget; the plan's exact bound is checked in the model's order, and if the
floating-point sum lands above tau the budget is shrunk by 2^-20 and the
table rebuilt (at most 8 times).

Best-first search (per-level interpolation with decomposition).  The
merged level-0 segments of max ordering form one unit whose steps are not
planes of one stream; the search takes its step counts s = 0, 1, ... in
order of their fetch cost (cheapest first), gives each the budget left after
its own exact error term, R - wd_0 * level_s, and lets the dynamic program
above spend that budget on the other units.  Pruning: positions whose own
term exceeds the budget are skipped, and the search stops at the first
position whose own cost is not below the best total found (every later one
costs more).  Ties go to the smaller s.
"""
from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from .plan import BelowFloor, Plan, bound, bound_for_planes, make_plan, plan_bytes, stream_planes

DP_PARTS = 2048
DP_RETRIES = 8


def _wd(grp, mode):
    return grp.wd_inf if mode == "inf" else grp.wd_2


def resident_steps(ref, resident: Optional[List[int]]) -> List[int]:
    """Steps of every unit covered by the resident planes of each stream."""
    if resident is None:
        return [0] * len(ref.units)
    out = []
    for unit in ref.units:
        if unit.kind == "plane":
            out.append(min(unit.meta.B, resident[unit.stream]))
        else:
            s = 0
            while s < len(unit.seg_steps) and all(p < resident[st] for st, p in unit.seg_steps[s]):
                s += 1
            out.append(s)
    return out


def step_cost(ref, u: int, k: int, resident: Optional[List[int]]) -> int:
    """Bytes of step k of unit u that are not resident."""
    unit = ref.units[u]
    if unit.kind == "plane":
        if resident is not None and k < resident[unit.stream]:
            return 0
        return unit.meta.plane_bytes(k)
    total = 0
    for st, p in unit.seg_steps[k]:
        if resident is None or p >= resident[st]:
            total += ref.streams[st].meta.plane_bytes(p)
    return total


def _extra_bytes(ref, planes: List[int], resident: Optional[List[int]]) -> int:
    total = 0
    for s, st in enumerate(ref.streams):
        lo = 0 if resident is None else resident[s]
        for j in range(lo, planes[s]):
            total += st.meta.plane_bytes(j)
    return total


def _as_plan(ref, planes: List[int], units: List[int], mode, resident, nsteps=None) -> Plan:
    """A plan from per-stream planes (resident planes kept: they cost
    nothing and only lower the error); its bound is the model's for exactly
    those planes; nsteps counts unit steps unless given."""
    if resident is not None:
        planes = [max(a, b) for a, b in zip(planes, resident)]
    return Plan(planes=list(planes), units=list(units), bound=bound_for_planes(ref, planes, mode),
                bytes=plan_bytes(ref, planes), nsteps=sum(units) if nsteps is None else nsteps)


def _greedy(ref, tau, mode, resident):
    pl = make_plan(ref, tau, mode)  # raises BelowFloor when no plan exists
    return _as_plan(ref, pl.planes, pl.units, mode, resident, nsteps=pl.nsteps)


def _budget(ref, tau, mode):
    const = ref.eps_fp
    for g in ref.group_order:
        const = const + _wd(ref.groups[g], mode) * 0.5
    return tau - const


def _dp_solve(ref, mode, units: List[int], R: float, k0: List[int], resident, parts: int):
    """Fewest bytes over the given units with their error terms, rounded up
    to parts of R / parts, summing to at most R: (bytes, {unit: steps}) or
    None when no choice fits."""
    if not (R > 0.0):
        return None
    q = R / parts
    # dp[b]: fewest bytes of the units so far whose parts sum to at most b
    # (bytes are integers below 2^53, exact in float64)
    dp = np.zeros(parts + 1)
    choice = []
    for u in units:
        unit = ref.units[u]
        wd = _wd(ref.groups[unit.group], mode)
        nd = np.full(parts + 1, np.inf)
        ch = np.full(parts + 1, -1, dtype=np.int64)
        parts_of = {}
        c = 0
        for k in range(k0[u], unit.nsteps + 1):
            if k > k0[u]:
                c += step_cost(ref, u, k - 1, resident)
            a = wd * float(unit.err(k))
            A = int(math.ceil(a / q)) if a > 0.0 else 0
            parts_of[k] = A
            if A > parts:
                continue
            v = np.full(parts + 1, np.inf)
            v[A:] = c + dp[:parts + 1 - A]
            better = v < nd  # ties keep the smaller step count
            nd = np.where(better, v, nd)
            ch = np.where(better, k, ch)
        dp = nd
        choice.append((u, ch, parts_of))
    if not np.isfinite(dp[parts]):
        return None
    steps = {}
    b = parts
    for u, ch, parts_of in reversed(choice):
        k = int(ch[b])
        steps[u] = k
        b -= parts_of[k]
    return int(dp[parts]), steps


def _better(ref, best, greedy, resident):
    if best is None or _extra_bytes(ref, best.planes, resident) > _extra_bytes(ref, greedy.planes, resident):
        return greedy
    return best


def dp_plan(ref, tau: float, mode: str, resident: Optional[List[int]] = None, parts: int = DP_PARTS) -> Plan:
    """Dynamic-programming interpreter (fewest bytes within the budget)."""
    greedy = _greedy(ref, tau, mode, resident)
    k0 = resident_steps(ref, resident)
    R = _budget(ref, tau, mode)
    best = None
    for _ in range(DP_RETRIES):
        sol = _dp_solve(ref, mode, list(range(len(ref.units))), R, k0, resident, parts)
        if sol is None:
            break
        state = [sol[1][u] for u in range(len(ref.units))]
        if bound(ref, state, mode) <= tau:
            best = _as_plan(ref, stream_planes(ref, state), state, mode, resident)
            break
        R = R * (1.0 - 2.0 ** -20)
    return _better(ref, best, greedy, resident)


def best_first_plan(ref, tau: float, mode: str, resident: Optional[List[int]] = None, parts: int = DP_PARTS) -> Plan:
    """Best-first search over the staircase's steps, the other units by the
    dynamic program (per-level interpolation with decomposition); without a
    staircase this is the dynamic program."""
    stairs = [u for u, unit in enumerate(ref.units) if unit.kind == "stair"]
    if not stairs:
        return dp_plan(ref, tau, mode, resident, parts)
    greedy = _greedy(ref, tau, mode, resident)
    su = stairs[0]
    stair = ref.units[su]
    others = [u for u in range(len(ref.units)) if u != su]
    k0 = resident_steps(ref, resident)
    wd0 = _wd(ref.groups[stair.group], mode)
    R0 = _budget(ref, tau, mode)
    # staircase positions with their own cost, cheapest first
    pos = []
    c = 0
    for s in range(k0[su], stair.nsteps + 1):
        if s > k0[su]:
            c += step_cost(ref, su, s - 1, resident)
        pos.append((c, s))
    pos.sort()
    best = None
    for _ in range(DP_RETRIES):
        found = None  # (total bytes, s, steps)
        for cost, s in pos:
            if found is not None and cost >= found[0]:
                break
            a = wd0 * float(stair.err(s))
            if a > R0:
                continue
            sol = _dp_solve(ref, mode, others, R0 - a, k0, resident, parts)
            if sol is None:
                continue
            if found is None or cost + sol[0] < found[0]:
                found = (cost + sol[0], s, sol[1])
        if found is None:
            break
        state = [0] * len(ref.units)
        for u, k in found[2].items():
            state[u] = k
        state[su] = found[1]
        if bound(ref, state, mode) <= tau:
            best = _as_plan(ref, stream_planes(ref, state), state, mode, resident)
            break
        R0 = R0 * (1.0 - 2.0 ** -20)
    return _better(ref, best, greedy, resident)


def paper_plan(ref, tau: float, mode: str, resident: Optional[List[int]] = None) -> Plan:
    """The paper's choice: dynamic programming for per-region interpolation,
    best-first search for per-level interpolation (which is the dynamic
    program when there is no staircase)."""
    if ref.scheme.kind == "region":
        return dp_plan(ref, tau, mode, resident)
    return best_first_plan(ref, tau, mode, resident)


__all__ = ["BelowFloor", "dp_plan", "best_first_plan", "paper_plan", "resident_steps", "step_cost"]
