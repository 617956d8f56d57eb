"""GPU retrievals planned by the paper's interpreters (dynamic program for
per-region, best-first search for per-level interpolation), invoked
incrementally along a sequence of targets on one handle, against the
oracle's interpreters with the same resident planes: plans, bytes and
reconstructions bit for bit."""
import numpy as np
import pytest

import fieldgen
import oracle
from oracle import interp
from oracle.pipeline import target_tau

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEQ = [("rel", 1e-2), ("psnr", 60), ("rel", 1e-5), ("rel", 1e-3), ("psnr", 100)]


def _apc():
    import paper_2609_04573_amd as apc
    return apc


@pytest.mark.parametrize("scheme", [("level", None, 0), ("region", (1, 2, 0), 1), ("region", None, None)], ids=str)
@pytest.mark.parametrize("name", ["paper", "dp"])
def test_incremental_interpreter_retrievals_match_oracle(config1_field, scheme, name):
    apc = _apc()
    kind, order, cd = scheme
    x = config1_field
    ref = oracle.refactor(x, oracle.Scheme(kind=kind, order=order, cd_axis=cd))
    h = apc.refactor(torch.from_numpy(x).cuda(), apc.Scheme(kind=kind, order=order, cd_axis=cd))
    h.set_interpreter(name)
    fn = interp.paper_plan if name == "paper" else interp.dp_plan
    resident = None
    for tk, tv in SEQ:
        tau, mode = target_tau(ref, oracle.Target(tk, tv))
        pl = fn(ref, tau, mode, resident)
        planes, info = h.plan(apc.Target(tk, tv))
        assert planes == pl.planes and info["bytes_total"] == pl.bytes and info["bound"] == pl.bound, (tk, tv)
        out, rinfo = h.retrieve(apc.Target(tk, tv))
        want = oracle.retrieve(ref, pl)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), want.view(np.uint32)), (tk, tv)
        resident = list(pl.planes) if resident is None else [max(a, b) for a, b in zip(resident, pl.planes)]
    h.close()


def test_ladder_with_the_paper_interpreter(config1_field):
    apc = _apc()
    x = config1_field
    ref = oracle.refactor(x, oracle.Scheme(kind="level", cd_axis=0))
    h = apc.refactor(torch.from_numpy(x).cuda(), apc.Scheme(kind="level", cd_axis=0))
    h.set_interpreter("paper")
    targets = [apc.Target("rel", r) for r in (1e-1, 1e-3, 1e-5)]
    lad = apc.Ladder(h, targets)
    outs = lad.launch()
    torch.cuda.synchronize()
    resident = None
    for t, o in zip(targets, outs):
        tau, mode = target_tau(ref, oracle.Target(t.kind, t.value))
        pl = interp.paper_plan(ref, tau, mode, resident)
        want = oracle.retrieve(ref, pl)
        assert np.array_equal(o.cpu().numpy().view(np.uint32), want.view(np.uint32)), t
        resident = list(pl.planes) if resident is None else [max(a, b) for a, b in zip(resident, pl.planes)]
    lad.close()
    h.close()
