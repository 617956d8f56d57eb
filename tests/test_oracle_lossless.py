"""Pins of the oracle's lossless stage (zero-word suppression of magnitude
planes): the hand-worked blob of tests/golden/lossless_stream.json, the
round trip against the generic blob at every plane count, the choice of raw
planes where suppression would not pay, and the retrieval path (same
reconstruction for the same planes, fewer or equal bytes, guarantees)."""
import json
import os

import numpy as np
import pytest

import fieldgen
import oracle
from oracle import bitplane
from oracle.plan import plan_bytes

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_hand_worked_lossless_blob():
    g = json.load(open(os.path.join(GOLD, "lossless_stream.json")))
    q = np.zeros(g["n"], dtype=np.int64)
    for i, v in g["codes"].items():
        q[int(i)] = v
    blob, meta = bitplane.encode(q, lossless=True)
    assert meta.B == g["B"] and meta.nnz == g["nnz"]
    assert [meta.suppressed(j) for j in range(meta.B)] == g["suppressed"]
    assert [meta.plane_bytes(j) for j in range(meta.B)] == g["plane_bytes"]
    words = [int(w, 16) for w in g["blob_words_after_index"]]
    assert blob == bytes(g["index_bytes"]) + np.array(words, dtype="<u8").tobytes()
    gen, gmeta = bitplane.encode(q)
    assert [gmeta.plane_bytes(j) for j in range(gmeta.B)] == g["generic_plane_bytes"]
    assert len(gen) == 280 and len(blob) == 120


@pytest.mark.parametrize("density", [0.0005, 0.01, 0.3, 1.0])
@pytest.mark.parametrize("n", [1, 63, 4097, 9000])
def test_round_trip_matches_generic_blob(density, n):
    rng = np.random.default_rng(int(density * 1e4) + n)
    q = np.where(rng.random(n) < density, rng.integers(-(1 << 20), 1 << 20, n), 0).astype(np.int64)
    blob, meta = bitplane.encode(q, lossless=True)
    gen, gmeta = bitplane.encode(q)
    assert meta.nsig == gmeta.nsig and meta.B == gmeta.B
    for k in range(meta.B + 1):
        got = bitplane.decode(blob, meta, k)
        assert np.array_equal(got, bitplane.decode(gen, gmeta, k))
        assert np.array_equal(got, bitplane.truncate(q, meta.B, k))
    for j in range(meta.B):
        assert meta.plane_bytes(j) <= gmeta.plane_bytes(j)
        assert bitplane.plane_words(blob, meta, j) == bitplane.plane_words(gen, gmeta, j)
    assert len(blob) == bitplane.section_offsets(meta)[2] + 8 * sum((v + 63) // 64 for v in meta.nsig)


def test_dense_planes_stay_raw():
    rng = np.random.default_rng(3)
    q = rng.integers(1, 1 << 12, 5000).astype(np.int64)  # every word of the low planes is nonzero
    blob, meta = bitplane.encode(q, lossless=True)
    assert not meta.suppressed(meta.B - 1)
    assert meta.nnz[meta.B - 1] == meta.words


@pytest.mark.parametrize("scheme", [("level", 0), ("region", None)], ids=str)
def test_retrieval_with_the_lossless_stage(scheme):
    kind, cd = scheme
    x = fieldgen.power_law_field((24, 40, 48), seed=13)
    plain = oracle.refactor(x, oracle.Scheme(kind=kind, cd_axis=cd))
    ll = oracle.refactor(x, oracle.Scheme(kind=kind, cd_axis=cd, lossless=True))
    def nseg(ref):
        return sum(len(u.seg_bytes) for u in ref.units if u.kind == "stair")

    # 4 more metadata bytes per plane (its nonzero word count); the staircase
    # may differ (it orders planes by error decrease per stored byte)
    assert (ll.meta_bytes - 8 * nseg(ll)
            == plain.meta_bytes - 8 * nseg(plain) + 4 * sum(st.meta.B for st in plain.streams))
    for rel in (1e-2, 1e-4, 1e-6):
        pl = oracle.plan(plain, oracle.Target("rel", rel))
        # the same planes reconstruct the same field from either blob
        assert np.array_equal(oracle.retrieve(ll, pl.planes).view(np.uint32),
                              oracle.retrieve(plain, pl.planes).view(np.uint32))
        pll = oracle.plan(ll, oracle.Target("rel", rel))
        out = oracle.retrieve(ll, pll)
        assert np.abs(out.astype(np.float64) - x).max() <= rel * ll.range
        same_planes = plan_bytes(ll, pl.planes)
        assert same_planes - ll.meta_bytes <= pl.bytes - plain.meta_bytes
    total_ll = sum(len(st.blob) for st in ll.streams)
    total = sum(len(st.blob) for st in plain.streams)
    assert total_ll < total
