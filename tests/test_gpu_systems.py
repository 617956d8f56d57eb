"""GPU tests of the systems layer: batched refactoring of uneven fields,
hipGraph-captured retrieval ladders, and target-driven pipeline selection
(Section VI-A) against the CPU oracle's vote."""
import numpy as np
import pytest

import fieldgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _apc():
    import paper_2609_04573_amd as apc
    return apc


def _fields():
    rng = np.random.default_rng(9)
    return [
        (fieldgen.power_law_field((17, 30, 45), seed=21), ("level", 3, None, 1)),
        (fieldgen.config1_field(), ("region", 3, (0, 2, 1), 0)),
        (fieldgen.power_law_field((37, 129), seed=22), ("level", 3, None, 0)),
        (np.cumsum(rng.standard_normal(1000)).astype(np.float32), ("region", 1, (0,), None)),
        (fieldgen.power_law_field((9, 9, 9), seed=23), ("level", 1, None, None)),
        (fieldgen.power_law_field((40, 33, 70), seed=24), ("region", 3, (2, 1, 0), 2)),
    ]


def test_batch_refactor_equals_single_and_oracle():
    apc = _apc()
    fs = _fields()
    xs = [torch.from_numpy(x).cuda() for x, _ in fs]
    schemes = [apc.Scheme(kind=k, degree=d, order=o, cd_axis=c) for _, (k, d, o, c) in fs]
    hb = apc.refactor_batch(xs, schemes)
    for i, ((x, (k, d, o, c)), h) in enumerate(zip(fs, hb)):
        hs = apc.refactor(xs[i], schemes[i])
        assert h.metadata() == hs.metadata(), i
        for s in range(h.num_streams):
            assert h.stream_blob(s) == hs.stream_blob(s), (i, s)
        ref = oracle.refactor(x, oracle.Scheme(kind=k, degree=d, order=o, cd_axis=c))
        for s, st in enumerate(ref.streams):
            assert h.stream_blob(s) == st.blob, (i, s)
        got, _ = h.retrieve(apc.Target("rel", 1e-4))
        want = oracle.retrieve(ref, oracle.plan(ref, oracle.Target("rel", 1e-4)))
        assert np.array_equal(got.cpu().numpy().view(np.uint32), want.view(np.uint32)), i
        hs.close()
        h.close()


def test_batch_of_many_fields_takes_long_runs_and_matches_the_oracle():
    """In a batch of sixteen fields each level is cut into fewer blocks than
    for a field alone: the large 2D fields are swept 32 rows to a block (the
    last run ragged), the thin 3D field's coarse levels are single planes.
    Streams and a reconstruction of every field equal the oracle's."""
    apc = _apc()
    rng = np.random.default_rng(31)
    fs = [(fieldgen.zonal_bands((2100, 1000), seed=3), ("level", 3, None, 0)),
          (fieldgen.power_law_field((1100, 2100), seed=4), ("level", 3, None, 1)),
          (fieldgen.power_law_field((3, 400, 500), seed=5), ("level", 3, None, 0))]
    for i in range(13):
        shape = tuple(int(v) for v in rng.integers(5, 48, size=3))
        fs.append((fieldgen.power_law_field(shape, seed=40 + i), ("level", 3, None, i % 3)))
    xs = [torch.from_numpy(x).cuda() for x, _ in fs]
    schemes = [apc.Scheme(kind=k, degree=d, order=o, cd_axis=c) for _, (k, d, o, c) in fs]
    hb = apc.refactor_batch(xs, schemes)
    for i, ((x, (k, d, o, c)), h) in enumerate(zip(fs, hb)):
        ref = oracle.refactor(x, oracle.Scheme(kind=k, degree=d, order=o, cd_axis=c))
        for s, st in enumerate(ref.streams):
            assert h.stream_blob(s) == st.blob, (i, s)
        got, _ = h.retrieve(apc.Target("rel", 1e-4))
        want = oracle.retrieve(ref, oracle.plan(ref, oracle.Target("rel", 1e-4)))
        assert np.array_equal(got.cpu().numpy().view(np.uint32), want.view(np.uint32)), i
        h.close()


def test_batch_of_float64_fields_with_single_plane_levels_matches_the_oracle():
    """float64 1D, 2D and thin 3D fields refactored in one batch (one-column
    sweep tiles, one-row decomposition slices) give the oracle's streams and
    reconstructions."""
    apc = _apc()
    fs = [(fieldgen.power_law_field((3900,), seed=51, dtype=np.float64), ("level", 3, None, None)),
          (fieldgen.power_law_field((300, 1100), seed=52, dtype=np.float64), ("level", 3, None, 0)),
          (fieldgen.power_law_field((2, 500, 600), seed=53, dtype=np.float64), ("level", 1, None, 0)),
          (fieldgen.power_law_field((130, 2050), seed=54, dtype=np.float64), ("region", 3, None, 0))]
    xs = [torch.from_numpy(x).cuda() for x, _ in fs]
    schemes = [apc.Scheme(kind=k, degree=d, order=o, cd_axis=c) for _, (k, d, o, c) in fs]
    hb = apc.refactor_batch(xs, schemes)
    for i, ((x, (k, d, o, c)), h) in enumerate(zip(fs, hb)):
        ref = oracle.refactor(x, oracle.Scheme(kind=k, degree=d, order=o, cd_axis=c))
        for s_, st in enumerate(ref.streams):
            assert h.stream_blob(s_) == st.blob, (i, s_)
        for t in (apc.Target("rel", 1e-3), apc.Target("psnr", 120)):
            got, _ = h.retrieve(t)
            want = oracle.retrieve(ref, oracle.plan(ref, oracle.Target(t.kind, t.value)))
            assert np.array_equal(got.cpu().numpy().view(np.uint64), want.view(np.uint64)), (i, t)
        h.close()


def test_batch_rejects_mixed_dtypes_and_bad_fields():
    apc = _apc()
    a = torch.zeros((8, 8, 8), device="cuda")
    b = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(AssertionError):
        apc.refactor_batch([a, b], [apc.Scheme(), apc.Scheme()])
    c = torch.zeros((8, 8, 8), device="cuda")
    c[0, 0, 0] = float("inf")
    with pytest.raises(apc.ApcError) as ei:
        apc.refactor_batch([a, c], [apc.Scheme(), apc.Scheme()])
    assert ei.value.status == -3


def test_ladder_graph_replays_match_single_shot(config1_field):
    apc = _apc()
    x = torch.from_numpy(config1_field).cuda()
    sc = apc.Scheme(kind="level", cd_axis=0)
    targets = [apc.Target("rel", r) for r in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6)] + [apc.Target("psnr", 70)]
    want = []
    for t in targets:
        fresh = apc.refactor(x, sc)
        out, _ = fresh.retrieve(t)
        want.append(out.clone())
        fresh.close()
    h = apc.refactor(x, sc)
    ladder = apc.Ladder(h, targets)
    other = apc.refactor(x, apc.Scheme(kind="region"))
    for rep in range(3):
        for o in ladder.outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        outs = ladder.launch()
        torch.cuda.synchronize()
        for i, (g, w) in enumerate(zip(outs, want)):
            assert torch.equal(g.view(torch.int32), w.view(torch.int32)), (rep, i)
        # eager work between replays: other retrievals and a torch reduction
        other.retrieve(apc.Target("rel", 1e-3))
        _ = (x * 2).sum().item()
        torch.cuda.synchronize()
    # after a replay the handle continues incrementally from the ladder's last planes
    got, _ = h.retrieve(apc.Target("rel", 1e-3))
    fresh = apc.refactor(x, sc)
    ref, _ = fresh.retrieve(apc.Target("rel", 1e-3))
    assert torch.equal(got.view(torch.int32), ref.view(torch.int32))
    ladder.close()
    other.close()
    fresh.close()
    h.close()


def test_ladder_and_static_retrieval_of_a_2d_field_match_the_oracle():
    """A 2D field's levels take one-column sweep tiles and its one-row
    decomposition slices are rebuilt eight to a tile; the same launches
    captured in a graph ladder (replayed twice, eager work between) and run
    from the static scratch give the oracle's reconstructions."""
    apc = _apc()
    x = fieldgen.zonal_bands((257, 2100), seed=8)
    ref = oracle.refactor(x, oracle.Scheme(kind="level", cd_axis=0))
    xd = torch.from_numpy(x).cuda()
    h = apc.refactor(xd, apc.Scheme(kind="level", cd_axis=0))
    targets = [apc.Target("rel", 1e-2), apc.Target("psnr", 70), apc.Target("rel", 1e-5)]
    wants = [oracle.retrieve(ref, oracle.plan(ref, oracle.Target(t.kind, t.value))) for t in targets]
    ladder = apc.Ladder(h, targets)
    for rep in range(2):
        outs = ladder.launch()
        torch.cuda.synchronize()
        for i, (o, w) in enumerate(zip(outs, wants)):
            assert np.array_equal(o.cpu().numpy().view(np.uint32), w.view(np.uint32)), (rep, i)
        _ = (xd * 2).sum().item()
    ladder.close()
    for t, w in zip(targets, wants):
        out, _ = h.retrieve_static(t)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), w.view(np.uint32)), t
    h.close()


@pytest.mark.parametrize("mode", ["eb", "psnr"])
def test_select_pipeline_matches_oracle(config1_field, mode):
    apc = _apc()
    got = apc.select_pipeline(torch.from_numpy(config1_field).cuda(), mode)
    want = oracle.select_pipeline(config1_field, mode)
    assert (got.kind, got.cd_axis) == (want.kind, want.cd_axis)
    if want.kind == "region":
        assert tuple(got.order) == tuple(want.order)


def test_select_pipeline_2d_matches_oracle():
    apc = _apc()
    x = fieldgen.zonal_bands((300, 600), seed=2)
    got = apc.select_pipeline(torch.from_numpy(x).cuda(), "eb")
    want = oracle.select_pipeline(x, "eb")
    assert (got.kind, got.cd_axis) == (want.kind, want.cd_axis)
    if want.kind == "region":
        assert tuple(got.order) == tuple(want.order)


def test_tile_widths_do_not_change_results(config1_field):
    """Every sweep tile width gives the oracle's streams and reconstructions;
    the autotuner picks one of them and records it for the level shape."""
    apc = _apc()
    fields = [config1_field, fieldgen.zonal_bands((130, 300), seed=5), fieldgen.power_law_field((33, 70, 150), seed=6)]
    try:
        for x in fields:
            sc = oracle.Scheme(kind="level", cd_axis=0)
            ref = oracle.refactor(x, sc)
            want = oracle.retrieve(ref, oracle.plan(ref, oracle.Target("rel", 1e-4)))
            xd = torch.from_numpy(x).cuda()
            for t2 in (32, 64, 128):
                apc.tile_override(t2)
                h = apc.refactor(xd, apc.Scheme(kind="level", cd_axis=0))
                for s, st in enumerate(ref.streams):
                    assert h.stream_blob(s) == st.blob, (x.shape, t2, s)
                got, _ = h.retrieve(apc.Target("rel", 1e-4))
                assert np.array_equal(got.cpu().numpy().view(np.uint32), want.view(np.uint32)), (x.shape, t2)
                h.close()
        apc.tile_override(0)
        big = torch.from_numpy(fieldgen.power_law_field((64, 128, 256), seed=7)).cuda()
        r = apc.tune_tiles(big)
        assert r["tile"] in (32, 64, 128)
        assert all(v > 0 for v in r["us"].values())
        assert apc.tile_width(torch.float32, 128, 256) == r["tile"]
        with pytest.raises(apc.ApcError):
            apc.tile_override(48)
    finally:
        apc.tile_override(0)


def test_two_stream_retrieval_equals_one_stream():
    """A retrieval of a per-level field with a decomposition runs its coarse
    levels on a helper stream beside the level-0 work; with every launch
    profiled it runs on one stream.  Both give the oracle's values, for a
    fresh decode and for an incremental one on the same handle."""
    apc = _apc()
    x = fieldgen.power_law_field((40, 72, 300), seed=9)
    sc = oracle.Scheme(kind="level", cd_axis=0)
    ref = oracle.refactor(x, sc)
    xd = torch.from_numpy(x).cuda()
    outs = {}
    for one_stream in (False, True):
        h = apc.refactor(xd, apc.Scheme(kind="level", cd_axis=0))
        apc.apc.profile_enable(one_stream)
        try:
            for rel in (1e-2, 1e-5):
                got, _ = h.retrieve(apc.Target("rel", rel))
                torch.cuda.synchronize()
                outs[(one_stream, rel)] = got.cpu().numpy().view(np.uint32)
        finally:
            apc.apc.profile_enable(False)
            apc.apc.profile_report()
        h.close()
    for rel in (1e-2, 1e-5):
        want = oracle.retrieve(ref, oracle.plan(ref, oracle.Target("rel", rel))).view(np.uint32)
        assert np.array_equal(outs[(False, rel)], want), rel
        assert np.array_equal(outs[(True, rel)], want), rel


def test_refactor_returns_before_its_last_kernels():
    """The refactor returns while its sign placement may still run; a
    retrieval on another stream and a blob export right after it wait for
    the handle's ready event, so both see the finished representation: the
    retrieval equals the oracle's and the blobs equal those exported after
    a full device synchronization."""
    apc = _apc()
    x = fieldgen.power_law_field((48, 96, 256), seed=12)
    sc = oracle.Scheme(kind="level", cd_axis=0)
    ref = oracle.refactor(x, sc)
    xd = torch.from_numpy(x).cuda()
    side = torch.cuda.Stream()
    h = apc.refactor(xd, apc.Scheme(kind="level", cd_axis=0))
    got, _ = h.retrieve(apc.Target("rel", 1e-4), stream=side)
    blobs = [h.stream_blob(s) for s in range(h.num_streams)]
    torch.cuda.synchronize()
    want = oracle.retrieve(ref, oracle.plan(ref, oracle.Target("rel", 1e-4))).view(np.uint32)
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want)
    assert blobs == [h.stream_blob(s) for s in range(h.num_streams)]
    h.close()


def test_auto_schemes_refactor_with_the_selected_pipeline():
    """APC_AUTO / APC_AUTO_PSNR: the refactor first runs the target-driven
    selection (Section VI-A) and then refactors with what it picked, keeping
    the requested lossless stage and encoding; the result is the same handle
    as refactoring with that scheme, and the oracle's selection agrees."""
    import paper_2609_04573_amd as apc

    x = fieldgen.power_law_field((64, 80, 96), seed=12)
    xd = torch.from_numpy(x).cuda()
    for kind, mode in (("auto", "eb"), ("auto_psnr", "psnr")):
        sel = apc.select_pipeline(xd, mode)
        want = oracle.select_pipeline(x, mode)
        assert sel.kind == want.kind and sel.cd_axis == want.cd_axis, (mode, sel, want)
        h = apc.refactor(xd, apc.Scheme(kind=kind, lossless=True, encoding="negabinary_xor"))
        got = h.scheme
        assert got.kind == sel.kind and got.cd_axis == sel.cd_axis and got.degree == sel.degree, (got, sel)
        assert got.lossless and got.encoding == "negabinary_xor"
        ref = apc.refactor(xd, apc.Scheme(kind=sel.kind, degree=sel.degree, order=sel.order, cd_axis=sel.cd_axis,
                                          lossless=True, encoding="negabinary_xor"))
        assert h.metadata() == ref.metadata()
        for s in range(h.num_streams):
            assert h.stream_blob(s) == ref.stream_blob(s)
        hb = apc.refactor_batch([xd, xd], [apc.Scheme(kind=kind), apc.Scheme(kind="level")])
        assert hb[0].scheme.kind == sel.kind and hb[1].scheme.kind == "level"
        for hh in [h, ref] + hb:
            hh.close()
