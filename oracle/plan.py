"""Retrieval interpreter: error model, max ordering and greedy plane selection
(Section V-C; Algorithm 2 "RetrievalInterpreter"; problem statements of
Section III-A).

Error model.  With Delta_g the quantization step of group g and e_g the
largest integer error left in its codes by the planes not fetched,

  E_inf = sum_g (w_g * Delta_g) * (0.5 + e_g) + eps_fp     (max-error bound)
  E_2   = sum_g (rho_g * Delta_g) * (0.5 + e_g) + eps_fp   (RMSE bound)

summed over groups in unit order.  e_g is delta_u(k_u) for a group with one
stream; the sum over S1, S2, S3 for a per-region group with coefficient
decomposition (the integer lifting adds errors at most); and the max over
regions of that sum for the finest per-level group with decomposition (regions
of one per-level level do not feed each other, Section V-C), tracked by the
staircase below.  eps_fp = u_out*A' + 2^-40*W*A' covers the final cast
(u_out = 2^-24 for float32, 2^-53 for float64) and float64 rounding, with
W = sum_g w_g and A' = max|x| + E_inf(no planes, without eps_fp).

Max ordering (Section V-C, per-level with decomposition).  Each region first
orders its S1/S2/S3 planes greedily by error decrease per byte (ties to the
lower stream).  The regions are then merged: every region whose current error
equals the current maximum takes its next plane, and those planes together
form one segment; the maximum strictly decreases from segment to segment and
the list of maxima is the segment -> error-bound metadata.

Greedy interpreter (the deterministic stand-in for the paper's best-first
search / dynamic programming, which the paper names but does not give).
Units are ordered coarsest group first, then levels L-2 .. 0, regions in
ascending order, streams S1..S3.  Starting from no planes: stop as soon as
E <= tau; otherwise advance the unit with the largest
((w_g*Delta_g) * decrease of e_g) / bytes of the step, ties to the lowest unit
index.  A step ends at the unit's next lower error: planes that do not lower
it (the first digit planes of a negabinary stream) go with the plane that
does, in the greedy order and in max ordering alike.  The order does not depend on tau, so plans for tighter targets
contain the plans for looser ones.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

from .bitplane import StreamMeta


class BelowFloor(Exception):
    """The requested target is tighter than the full representation allows."""


@dataclass
class Unit:
    group: int
    kind: str                        # "plane" or "stair"
    stream: int = -1                 # plane unit: its stream
    meta: Optional[StreamMeta] = None
    levels: List[int] = field(default_factory=list)      # stair: max error after j segments
    seg_bytes: List[int] = field(default_factory=list)   # stair: bytes of segment j
    seg_steps: List[list] = field(default_factory=list)  # stair: [(stream, plane)] per segment

    @property
    def nsteps(self) -> int:
        return self.meta.B if self.kind == "plane" else len(self.seg_bytes)

    def err(self, k: int) -> int:
        return self.meta.delta(k) if self.kind == "plane" else self.levels[k]

    def step_bytes(self, k: int) -> int:
        return self.meta.plane_bytes(k) if self.kind == "plane" else self.seg_bytes[k]


def next_lower(err, k: int, n: int) -> int:
    """The first step count after k whose error is below err(k) (n at most).
    Steps that do not lower the error (the first digit planes of a
    negabinary stream) are taken together with the step that does."""
    k2 = k + 1
    while k2 < n and err(k2) >= err(k):
        k2 += 1
    return k2


def build_staircase(group: int, region_streams: List[List[int]], metas: List[StreamMeta]) -> Unit:
    """Max ordering over the regions of the finest per-level level."""
    orders = []
    for trip in region_streams:
        k = [0, 0, 0]
        steps = []  # (stream t, planes taken together)
        while True:
            best, best_r, best_n = -1, -1.0, 0
            for t in range(3):
                m = metas[trip[t]]
                if k[t] < m.B:
                    k2 = next_lower(m.delta, k[t], m.B)
                    gain = m.delta(k[t]) - m.delta(k2)
                    nb = sum(m.plane_bytes(j) for j in range(k[t], k2))
                    r = float(gain) / float(nb)
                    if r > best_r:
                        best, best_r, best_n = t, r, k2 - k[t]
            if best < 0:
                break
            steps.append((best, best_n))
            k[best] += best_n
        orders.append(steps)

    R = len(region_streams)
    pos = [0] * R
    kk = [[0, 0, 0] for _ in range(R)]

    def err(r: int) -> int:
        return sum(metas[region_streams[r][t]].delta(kk[r][t]) for t in range(3))

    e = [err(r) for r in range(R)]
    unit = Unit(group=group, kind="stair")
    unit.levels.append(max(e) if R else 0)
    while unit.levels[-1] > 0:
        top = unit.levels[-1]
        nb = 0
        steps = []
        for r in range(R):
            if e[r] == top:
                t, cnt = orders[r][pos[r]]
                pos[r] += 1
                u = region_streams[r][t]
                for _ in range(cnt):
                    nb += metas[u].plane_bytes(kk[r][t])
                    steps.append((u, kk[r][t]))
                    kk[r][t] += 1
                e[r] = err(r)
        unit.levels.append(max(e))
        unit.seg_bytes.append(nb)
        unit.seg_steps.append(steps)
    return unit


def group_error(ref, g: int, state: List[int]) -> int:
    us = ref.group_units[g]
    if len(us) == 1:
        return ref.units[us[0]].err(state[us[0]])
    return sum(ref.units[u].err(state[u]) for u in us)


def bound(ref, state: List[int], mode: str) -> float:
    E = 0.0
    for g in ref.group_order:
        grp = ref.groups[g]
        wd = grp.wd_inf if mode == "inf" else grp.wd_2
        E = E + wd * (0.5 + group_error(ref, g, state))
    return E + ref.eps_fp


def eps_fp(ref) -> float:
    zero = [0] * len(ref.units)
    e0 = 0.0
    W = 0.0
    for g in ref.group_order:
        grp = ref.groups[g]
        e0 = e0 + grp.wd_inf * (0.5 + group_error(ref, g, zero))
        W = W + grp.w
    Ap = ref.A + e0
    u_out = 2.0 ** -24 if ref.P == 29 else 2.0 ** -53
    return u_out * Ap + (2.0 ** -40 * W) * Ap


def greedy_sequence(ref, mode: str):
    """Full greedy order: list of (unit advanced, its step count after the
    step, bound after the step).  A step runs to the unit's next lower error
    (one step, except for negabinary digit planes that do not lower it)."""
    state = [0] * len(ref.units)
    seq = []
    E0 = bound(ref, state, mode)
    while True:
        best, best_s, best_k = -1, -1.0, 0
        for u, unit in enumerate(ref.units):
            if state[u] < unit.nsteps:
                grp = ref.groups[unit.group]
                wd = grp.wd_inf if mode == "inf" else grp.wd_2
                k = state[u]
                k2 = next_lower(unit.err, k, unit.nsteps)
                de = unit.err(k) - unit.err(k2)
                s = (wd * float(de)) / float(sum(unit.step_bytes(j) for j in range(k, k2)))
                if s > best_s:
                    best, best_s, best_k = u, s, k2
        if best < 0:
            break
        state[best] = best_k
        seq.append((best, best_k, bound(ref, state, mode)))
    return E0, seq


@dataclass
class Plan:
    planes: List[int]      # planes per stream
    units: List[int]       # steps per unit
    bound: float
    bytes: int
    nsteps: int


def stream_planes(ref, ustate: List[int]) -> List[int]:
    k = [0] * len(ref.streams)
    for u, unit in enumerate(ref.units):
        if unit.kind == "plane":
            k[unit.stream] = ustate[u]
        else:
            for j in range(ustate[u]):
                for (s, plane) in unit.seg_steps[j]:
                    k[s] = max(k[s], plane + 1)
    return k


def plan_bytes(ref, k: List[int]) -> int:
    total = ref.meta_bytes
    for s, st in enumerate(ref.streams):
        for j in range(k[s]):
            total += st.meta.plane_bytes(j)
    return total


def make_plan(ref, tau: float, mode: str) -> Plan:
    if not (tau > 0.0):
        raise BelowFloor("target tolerance must be positive")
    E0, seq = ref.sequence(mode)
    state = [0] * len(ref.units)
    E = E0
    n = 0
    while E > tau:
        if n == len(seq):
            raise BelowFloor(f"tau={tau!r} below the floor {E!r}")
        u, k, E = seq[n]
        state[u] = k
        n += 1
    k = stream_planes(ref, state)
    return Plan(planes=k, units=state, bound=E, bytes=plan_bytes(ref, k), nsteps=n)


def bound_for_planes(ref, k: List[int], mode: str) -> float:
    """Bound of the model for any per-stream plane vector (not only greedy
    prefixes): a staircase group takes the max over its regions of the summed
    stream errors."""
    E = 0.0
    for g in ref.group_order:
        grp = ref.groups[g]
        wd = grp.wd_inf if mode == "inf" else grp.wd_2
        us = ref.group_units[g]
        if len(us) == 1 and ref.units[us[0]].kind == "stair":
            unit = ref.units[us[0]]
            per_region = {}
            for s, st in enumerate(ref.streams):
                if st.group == g:
                    per_region.setdefault(st.key[2], 0)
                    per_region[st.key[2]] += st.meta.delta(k[s])
            e = max(per_region.values()) if per_region else 0
        else:
            e = sum(ref.streams[ref.units[u].stream].meta.delta(k[ref.units[u].stream]) for u in us)
        E = E + wd * (0.5 + e)
    return E + ref.eps_fp
