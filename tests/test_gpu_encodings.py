"""GPU tests of the lossless stage and the negabinary encodings on the paths
that share launches or capture them: a batched refactor of fields with
different encodings, a retrieval ladder replayed as one graph, the serving
loop merging requests of differently encoded fields, the retrieval that
allocates nothing, and batched retrieval (repeated handles included).  Streams, plans and reconstructions must equal the
oracle's bit for bit (Table I encodings; Section V lossless stage)."""
import numpy as np
import pytest

import fieldgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (kind, degree, order, cd_axis, lossless, encoding)
CASES = [
    ("level", 3, None, 0, True, "generic"),
    ("region", 3, (2, 1, 0), None, False, "negabinary_xor"),
    ("level", 3, None, None, True, "negabinary"),
    ("region", 1, (0, 2, 1), 1, True, "negabinary_xor"),
]


def _apc():
    import paper_2609_04573_amd as apc
    return apc


def _schemes(case):
    apc = _apc()
    kind, degree, order, cd, ll, enc = case
    return (apc.Scheme(kind=kind, degree=degree, order=order, cd_axis=cd, lossless=ll, encoding=enc),
            oracle.Scheme(kind=kind, degree=degree, order=order, cd_axis=cd, lossless=ll, encoding=enc))


def _bits(a):
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


@pytest.fixture(scope="module")
def fields():
    shapes = [(40, 48, 56), (33, 40, 64), (48, 48, 48), (37, 45, 52)]
    xs = [fieldgen.power_law_field(s, seed=30 + i) for i, s in enumerate(shapes)]
    refs = [oracle.refactor(x, _schemes(c)[1]) for x, c in zip(xs, CASES)]
    return xs, refs


def _targets():
    apc = _apc()
    return [apc.Target("rel", 1e-2), apc.Target("psnr", 60), apc.Target("rel", 1e-4), apc.Target("psnr", 90)]


def test_batched_refactor_of_mixed_encodings(fields):
    apc = _apc()
    xs, refs = fields
    hs = apc.refactor_batch([torch.from_numpy(x).cuda() for x in xs], [_schemes(c)[0] for c in CASES])
    for f, (h, ref) in enumerate(zip(hs, refs)):
        for s, st in enumerate(ref.streams):
            assert h.stream_blob(s) == st.blob, (f, s)
        for t in _targets():
            out, info = h.retrieve(t)
            pl = oracle.plan(ref, oracle.Target(t.kind, t.value))
            assert info["bytes_total"] == pl.bytes, (f, t)
            want = oracle.retrieve(ref, pl)
            assert np.array_equal(_bits(out.cpu().numpy()), _bits(want)), (f, t)
        h.close()


def test_graph_ladder_on_negabinary_and_lossless_fields(fields):
    """Each ladder is replayed twice, with eager retrievals of the same handle
    in between; every replay must give the oracle's reconstructions."""
    apc = _apc()
    xs, refs = fields
    for f in (1, 3):
        h = apc.refactor(torch.from_numpy(xs[f]).cuda(), _schemes(CASES[f])[0])
        ts = _targets()
        lad = apc.Ladder(h, ts)
        wants = [oracle.retrieve(refs[f], oracle.plan(refs[f], oracle.Target(t.kind, t.value))) for t in ts]
        for rep in range(2):
            outs = lad.launch()
            torch.cuda.synchronize()
            for t, o, w in zip(ts, outs, wants):
                assert np.array_equal(_bits(o.cpu().numpy()), _bits(w)), (f, rep, t)
            eager, _ = h.retrieve(ts[rep])
            assert np.array_equal(_bits(eager.cpu().numpy()), _bits(wants[rep])), (f, rep)
        lad.close()
        h.close()


@pytest.mark.timeout(600)
def test_server_merges_requests_of_differently_encoded_fields(fields):
    apc = _apc()
    xs, refs = fields
    hs = [apc.refactor(torch.from_numpy(x).cuda(), _schemes(c)[0]) for x, c in zip(xs, CASES)]
    srv = apc.Server(hs, budget_bytes=4 << 30, max_slots=2, max_batch=8)
    rng = np.random.default_rng(5)
    reqs = []
    for _ in range(32):
        f = int(rng.integers(0, len(hs)))
        if rng.random() < 0.5:
            reqs.append((f, apc.Target("rel", float(rng.choice((1e-2, 1e-3, 1e-4, 1e-5))))))
        else:
            reqs.append((f, apc.Target("psnr", float(rng.choice((40, 60, 80, 100))))))
    outs = [torch.empty(xs[f].shape, dtype=torch.float32, device="cuda") for f, _ in reqs]
    tickets = [srv.submit(f, t, o) for (f, t), o in zip(reqs, outs)]
    for tk in tickets:
        srv.wait(tk)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["max_running"] >= 2, st
    for (f, t), o in zip(reqs, outs):
        want = oracle.retrieve(refs[f], oracle.plan(refs[f], oracle.Target(t.kind, t.value)))
        assert np.array_equal(_bits(o.cpu().numpy()), _bits(want)), (f, t)
    for h in hs:
        h.close()


def test_static_retrieval_of_negabinary_and_lossless_fields(fields):
    apc = _apc()
    xs, refs = fields
    for f in range(len(CASES)):
        h = apc.refactor(torch.from_numpy(xs[f]).cuda(), _schemes(CASES[f])[0])
        for t in _targets()[:2]:
            out, info = h.retrieve_static(t)
            pl = oracle.plan(refs[f], oracle.Target(t.kind, t.value))
            assert info["bytes_total"] == pl.bytes
            assert np.array_equal(_bits(out.cpu().numpy()), _bits(oracle.retrieve(refs[f], pl))), (f, t)
        h.close()


def test_batched_retrieval_equals_single_retrievals_and_the_oracle(fields):
    """apc_retrieve_batch over the differently encoded fields, a handle
    repeated with tighter and looser targets: every output equals the
    oracle's reconstruction for its plan, plans and byte counts equal the
    oracle's, and a later single retrieval continues from the planes the
    batch decoded."""
    apc = _apc()
    xs, refs = fields
    hs = [apc.refactor(torch.from_numpy(x).cuda(), _schemes(c)[0]) for x, c in zip(xs, CASES)]
    reqs = [(0, apc.Target("rel", 1e-4)), (1, apc.Target("psnr", 70)), (0, apc.Target("rel", 1e-2)),
            (2, apc.Target("rel", 1e-3)), (3, apc.Target("psnr", 90)), (0, apc.Target("rel", 1e-5)),
            (1, apc.Target("psnr", 50))]
    outs, infos = apc.retrieve_batch([hs[f] for f, _ in reqs], [t for _, t in reqs])
    kcur = {f: [0] * len(refs[f].streams) for f in range(len(hs))}
    for (f, t), o, inf in zip(reqs, outs, infos):
        pl = oracle.plan(refs[f], oracle.Target(t.kind, t.value))
        assert inf["bytes_total"] == pl.bytes, (f, t)
        added = 0
        for s, st in enumerate(refs[f].streams):
            for j in range(kcur[f][s], pl.planes[s]):
                added += st.meta.plane_bytes(j)
            kcur[f][s] = max(kcur[f][s], pl.planes[s])
        assert inf["bytes_fetched"] == added, (f, t)
        want = oracle.retrieve(refs[f], pl)
        assert np.array_equal(_bits(o.cpu().numpy()), _bits(want)), (f, t)
    # what the batch decoded stays resident: a looser single retrieval fetches nothing
    out, inf = hs[0].retrieve(apc.Target("rel", 1e-3))
    assert inf["bytes_fetched"] == 0
    pl = oracle.plan(refs[0], oracle.Target("rel", 1e-3))
    assert np.array_equal(_bits(out.cpu().numpy()), _bits(oracle.retrieve(refs[0], pl)))
    with pytest.raises(apc.BelowFloor):
        apc.retrieve_batch([hs[0], hs[1]], [apc.Target("rel", 1e-2), apc.Target("abs", 0.0)])
    for h in hs:
        h.close()


def test_batched_retrieval_of_float64_fields_of_every_dimensionality():
    """float64 fields of 1, 2 and 3 dims (tiny and ragged ones included) in
    one batched retrieval, a field repeated, against the oracle."""
    apc = _apc()
    rng = np.random.default_rng(8)
    shapes = [(1,), (2,), (3, 3), (700,), (45, 61), (9, 17, 30)]
    schemes = [("level", 3, None, None, False, "generic"), ("region", 1, None, None, True, "generic"),
               ("level", 3, None, 1, False, "negabinary_xor"), ("region", 3, None, None, True, "negabinary"),
               ("level", 3, None, 0, True, "generic"), ("region", 3, (1, 2, 0), 2, False, "negabinary_xor")]
    xs = [np.cumsum(rng.standard_normal(s), axis=-1).astype(np.float64) for s in shapes]
    hs, refs = [], []
    for x, c in zip(xs, schemes):
        kind, degree, order, cd, ll, enc = c
        if order is not None and len(order) != x.ndim:
            order = None
        gs = apc.Scheme(kind=kind, degree=degree, order=order, cd_axis=cd, lossless=ll, encoding=enc)
        osc = oracle.Scheme(kind=kind, degree=degree, order=order, cd_axis=cd, lossless=ll, encoding=enc)
        hs.append(apc.refactor(torch.from_numpy(x).cuda(), gs))
        refs.append(oracle.refactor(x, osc))
    reqs = [(f, apc.Target("abs", 1e-3)) for f in range(len(xs))] + [(4, apc.Target("psnr", 80)),
                                                                      (5, apc.Target("rel", 1e-6))]
    outs, infos = apc.retrieve_batch([hs[f] for f, _ in reqs], [t for _, t in reqs])
    for (f, t), o, inf in zip(reqs, outs, infos):
        pl = oracle.plan(refs[f], oracle.Target(t.kind, t.value))
        assert inf["bytes_total"] == pl.bytes, (f, t)
        want = oracle.retrieve(refs[f], pl)
        assert np.array_equal(_bits(o.cpu().numpy()), _bits(want)), (f, t)
    for h in hs:
        h.close()
