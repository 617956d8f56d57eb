"""The scale workload's path at a size the oracle finishes in a minute: a
256^3 float32 k^-5/3 field with ~1% sharp-front spheres (tanh steps of width
2 cells), seed 4.  Target-driven selection (Section VI-A) in both modes must
pick the oracle's scheme; the field refactored with the error-bound choice
must give the oracle's streams; the relative-eb ladder replayed as one graph
and a mixed eb / PSNR batch through the server must give the oracle's
reconstructions bit for bit."""
import numpy as np
import pytest

import fieldgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _apc():
    import paper_2609_04573_amd as apc
    return apc


@pytest.fixture(scope="module")
def fronts():
    return fieldgen.sharp_fronts((256, 256, 256), seed=4)


def _same(a, b):
    return a.kind == b.kind and a.cd_axis == b.cd_axis and (a.kind == "level" or tuple(a.order) == tuple(b.order))


@pytest.mark.timeout(600)
def test_sharp_fronts_selection_refactor_ladder_and_mixed_batch(fronts):
    apc = _apc()
    x = fronts
    xd = torch.from_numpy(x).cuda()
    sel = {}
    for mode in ("eb", "psnr"):
        got = apc.select_pipeline(xd, mode)
        want = oracle.select_pipeline(x, mode)
        assert _same(got, want), (mode, got, want)
        sel[mode] = want
    sc = sel["eb"]
    ref = oracle.refactor(x, sc)
    h = apc.refactor(xd, apc.Scheme(kind=sc.kind, degree=sc.degree, order=sc.order, cd_axis=sc.cd_axis))
    for s, st in enumerate(ref.streams):
        assert h.stream_blob(s) == st.blob, f"stream {s}"
    ladder = [apc.Target("rel", r) for r in (1e-1, 1e-2, 1e-3, 1e-4)]
    lad = apc.Ladder(h, ladder)
    outs = lad.launch()
    torch.cuda.synchronize()
    mixed = [("rel", 1e-2), ("psnr", 60), ("rel", 1e-5), ("psnr", 90)]
    srv = apc.Server([h], budget_bytes=8 << 30, max_slots=4)
    souts = [torch.empty_like(xd) for _ in mixed]
    tickets = [srv.submit(0, apc.Target(k, v), o) for (k, v), o in zip(mixed, souts)]
    for tk in tickets:
        srv.wait(tk)
    srv.close()
    lad.close()
    for t, o in list(zip([("rel", r.value) for r in ladder], outs)) + list(zip(mixed, souts)):
        pl = oracle.plan(ref, oracle.Target(*t))
        want = oracle.retrieve(ref, pl)
        assert np.array_equal(o.cpu().numpy().view(np.uint32), want.view(np.uint32)), t
    h.close()
