"""Pins of the oracle's dynamic-programming and best-first interpreters
(Section V-C; Algorithm 2): the hand-worked optimum of the greedy toy
(tests/golden/greedy_toy.json), brute force over every plan of small
refactorings at reduced precision (the interpreters are never below the
optimum, never above the greedy plan, always within the target, and the
dynamic program reaches the optimum whenever the optimum's rounded error
parts fit its budget), and incremental invocation (resident planes cost
nothing and are kept)."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import interp
from oracle.plan import BelowFloor, bound, make_plan, plan_bytes, stream_planes

from test_oracle_pins import _toy_ref

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_dp_finds_the_hand_worked_optimum():
    g = json.load(open(os.path.join(GOLD, "greedy_toy.json")))
    ref = _toy_ref(g)
    o = g["optimal"]
    for fn in (interp.dp_plan, interp.best_first_plan, interp.paper_plan):
        pl = fn(ref, o["tau"], "inf")
        assert pl.planes == o["planes"] and pl.bytes == o["bytes"] and pl.bound == o["bound"], fn.__name__
    assert make_plan(ref, o["tau"], "inf").bytes == 160
    with pytest.raises(BelowFloor):
        interp.dp_plan(ref, g["below_floor_tau"], "inf")


def _brute(ref, tau, mode):
    """Fewest bytes over every unit-step vector within tau (and its state)."""
    best = None
    for state in itertools.product(*[range(u.nsteps + 1) for u in ref.units]):
        state = list(state)
        if bound(ref, state, mode) <= tau:
            b = plan_bytes(ref, stream_planes(ref, state))
            if best is None or b < best[0]:
                best = (b, state)
    return best


CASES = [
    ((9, 9), oracle.Scheme(kind="level", cd_axis=0), 3),
    ((5, 5), oracle.Scheme(kind="region", order=(0, 1), cd_axis=1), 2),
    ((5, 9), oracle.Scheme(kind="region", order=(0, 1), cd_axis=1), 2),
    ((4, 5, 6), oracle.Scheme(kind="region", order=(2, 0, 1)), 2),
    ((33,), oracle.Scheme(kind="level"), 3),
    ((6, 13), oracle.Scheme(kind="level", degree=1), 3),
    ((5, 5, 5), oracle.Scheme(kind="level", cd_axis=2), 2),
]


@pytest.mark.parametrize("shape,scheme,P", CASES, ids=lambda c: str(c))
def test_interpreters_against_brute_force(shape, scheme, P):
    rng = np.random.default_rng(17)
    x = rng.standard_normal(shape)
    ref = oracle.refactor(x, scheme, precision=P)
    space = math.prod(u.nsteps + 1 for u in ref.units)
    assert space <= 200000, space
    for mode in ("inf", "l2"):
        E0 = bound(ref, [0] * len(ref.units), mode)
        Efull = bound(ref, [u.nsteps for u in ref.units], mode)
        for frac in (0.9, 0.5, 0.2, 0.05):
            tau = Efull + frac * (E0 - Efull)
            opt = _brute(ref, tau, mode)
            greedy = make_plan(ref, tau, mode)
            for fn in (interp.dp_plan, interp.best_first_plan):
                pl = fn(ref, tau, mode)
                assert pl.bound <= tau
                assert opt[0] <= pl.bytes <= greedy.bytes, (fn.__name__, mode, frac, opt[0], pl.bytes, greedy.bytes)
            # the dynamic program reaches the optimum when its rounded parts fit
            R = interp._budget(ref, tau, mode)
            q = R / interp.DP_PARTS
            parts = 0
            for u, unit in enumerate(ref.units):
                wd = ref.groups[unit.group].wd_inf if mode == "inf" else ref.groups[unit.group].wd_2
                a = wd * float(unit.err(opt[1][u]))
                parts += math.ceil(a / q) if a > 0.0 else 0
            if parts <= interp.DP_PARTS:
                assert interp.dp_plan(ref, tau, mode).bytes == opt[0]


def test_incremental_invocation_keeps_resident_planes_free():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((17, 20))
    ref = oracle.refactor(x, oracle.Scheme(kind="level", cd_axis=0))
    tau1, tau2 = 1e-2 * ref.range, 1e-4 * ref.range
    for fn in (interp.dp_plan, interp.best_first_plan):
        first = fn(ref, tau1, "inf")
        second = fn(ref, tau2, "inf", resident=first.planes)
        assert all(b >= a for a, b in zip(first.planes, second.planes))
        assert second.bound <= tau2
        fresh = fn(ref, tau2, "inf")
        extra = sum(st.meta.plane_bytes(j) for s, st in enumerate(ref.streams)
                    for j in range(first.planes[s], second.planes[s]))
        assert extra <= plan_bytes(ref, fresh.planes) - ref.meta_bytes
        # a target the resident planes already meet fetches nothing
        again = fn(ref, tau1, "inf", resident=second.planes)
        assert again.planes == second.planes
