"""Pins of the oracle's negabinary encoding (Table I, PSNR mode): the
hand-worked digit planes, XOR chaining and bounds of
tests/golden/negabinary_stream.json, the truncation bound checked
exhaustively for small maxima, round trips at every plane count (with and
without XOR and the lossless stage), and retrieval guarantees in both modes."""
import json
import math
import os

import numpy as np
import pytest

import fieldgen
import oracle
from oracle import bitplane

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_hand_worked_negabinary_stream():
    g = json.load(open(os.path.join(GOLD, "negabinary_stream.json")))
    q = np.array(g["codes"], dtype=np.int64)
    for xor, key in ((False, "planes"), (True, "xor_planes")):
        blob, meta = bitplane.encode_nb(q, xor=xor)
        assert meta.B == g["B"]
        assert np.frombuffer(blob, "<u8").tolist() == g[key]
        assert [meta.delta(k) for k in range(meta.B + 1)] == g["delta"]
        assert bitplane.decode(blob, meta, 2).tolist() == g["after_2_planes"]
        assert meta.plane_bytes(0) == 8  # digit planes only
    for v, n in g["digits"].items():
        assert bitplane.nb_digits(int(v)) == n


def test_truncation_bound_exhaustive():
    for V in range(0, 200):
        B = bitplane.nb_digits(V)
        q = np.arange(-V, V + 1, dtype=np.int64)
        w = bitplane.to_negabinary(q, B)
        assert (w >= 0).all() and (w < (1 << B)).all()
        assert np.array_equal(bitplane.from_negabinary(w, B), q)
        for k in range(B + 1):
            err = np.abs(q - bitplane.truncate_nb(q, B, k)).max()
            bound = V if k == 0 else bitplane.nb_delta(B, k)
            assert err <= bound, (V, k)
        if B:
            # the bound is reached for some value in range once two digits are dropped
            assert np.abs(q - bitplane.truncate_nb(q, B, B - 2)).max() <= bitplane.nb_delta(B, B - 2)


@pytest.mark.parametrize("xor", [False, True])
@pytest.mark.parametrize("lossless", [False, True])
@pytest.mark.parametrize("n,density", [(1, 1.0), (100, 0.5), (5000, 0.02), (9000, 1.0)])
def test_round_trip(xor, lossless, n, density):
    rng = np.random.default_rng(n + int(xor) + 2 * int(lossless))
    q = np.where(rng.random(n) < density, rng.integers(-(1 << 30), 1 << 30, n), 0).astype(np.int64)
    blob, meta = bitplane.encode_nb(q, xor=xor, lossless=lossless)
    for k in range(meta.B + 1):
        assert np.array_equal(bitplane.decode(blob, meta, k), bitplane.truncate_nb(q, meta.B, k)), k
    assert len(blob) == sum(meta.mag_bytes(j) for j in range(meta.B))


@pytest.mark.parametrize("scheme", [("region", None, "negabinary_xor", True), ("region", 1, "negabinary", False),
                                    ("level", 0, "negabinary_xor", False)], ids=str)
def test_retrieval_guarantees(config1_field, scheme):
    kind, cd, enc, ll = scheme
    x = config1_field
    ref = oracle.refactor(x, oracle.Scheme(kind=kind, cd_axis=cd, encoding=enc, lossless=ll))
    xf = x.astype(np.float64)
    for rel in (1e-2, 1e-4, 1e-6):
        pl = oracle.plan(ref, oracle.Target("rel", rel))
        assert np.abs(oracle.retrieve(ref, pl).astype(np.float64) - xf).max() <= rel * ref.range
    for p in (40, 70, 100):
        pl = oracle.plan(ref, oracle.Target("psnr", p))
        err = oracle.retrieve(ref, pl).astype(np.float64) - xf
        assert 20 * math.log10(ref.range / math.sqrt(np.mean(err ** 2))) >= p
    full = [st.meta.B for st in ref.streams]
    assert np.array_equal(oracle.retrieve(ref, full), oracle.pipeline.quantized_field(ref))
    generic = oracle.refactor(x, oracle.Scheme(kind=kind, cd_axis=cd))
    assert np.array_equal(oracle.pipeline.quantized_field(generic), oracle.pipeline.quantized_field(ref))
