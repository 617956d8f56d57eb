"""Out-of-core blocks: a host-resident field refactored block by block (the
paper's independent fixed-size blocks), each block's serialized
representation equal to the oracle's refactoring of that block written in
the same layout, and retrievals (only the planned planes of each block
uploaded) equal to the oracle's reconstruction of every block for the
absolute bound the target implies, with the bound holding overall."""
import math

import numpy as np
import pytest

import fieldgen
import oracle
from oracle.pipeline import target_tau

from test_serialize import oracle_bytes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _apc():
    import paper_2609_04573_amd as apc
    return apc


def _blocks(shape, block):
    nb = [(n + b - 1) // b for n, b in zip(shape, block)]
    for idx in np.ndindex(*nb):
        yield tuple(slice(i * b, min(n, (i + 1) * b)) for i, b, n in zip(idx, block, shape))


@pytest.mark.parametrize("case", [
    ((70, 90, 100), (32, 48, 64), oracle.Scheme(kind="level", cd_axis=0), np.float32, 3 << 20),
    ((70, 90, 100), (40, 40, 40), oracle.Scheme(kind="region", order=(2, 1, 0), lossless=True), np.float32, 1 << 40),
    ((130, 257), (64, 100), oracle.Scheme(kind="level", cd_axis=1, encoding="negabinary_xor"), np.float64, 1 << 40),
], ids=["level-cd0-small-groups", "region-lossless", "2d-negabinary-f64"])
def test_blocks_match_the_oracle_block_by_block(case):
    apc = _apc()
    shape, block, sc, dtype, group = case
    x = fieldgen.power_law_field(shape, seed=41, dtype=dtype)
    bs = apc.BlockSet(x, block, apc.Scheme(kind=sc.kind, degree=sc.degree, order=sc.order, cd_axis=sc.cd_axis,
                                          lossless=sc.lossless, encoding=sc.encoding), group_bytes=group)
    info = bs.info()
    refs = []
    for b, sl in enumerate(_blocks(shape, block)):
        ref = oracle.refactor(np.ascontiguousarray(x[sl]), sc)
        assert bs.blob(b) == oracle_bytes(ref), f"block {b}"
        refs.append((sl, ref))
    assert info["blocks"] == len(refs)
    assert info["xmin"] == float(x.min()) and info["xmax"] == float(x.max())
    rng = float(x.max()) - float(x.min())
    bits = np.uint32 if dtype == np.float32 else np.uint64
    for kind, val in (("rel", 1e-2), ("rel", 1e-5), ("psnr", 70)):
        out, rinfo = bs.retrieve(apc.Target(kind, val))
        want = np.empty_like(x)
        total = 0
        abs_t = oracle.Target("abs", val * rng) if kind == "rel" else oracle.Target("rmse", rng * 10 ** (-val / 20))
        for sl, ref in refs:
            pl = oracle.plan(ref, abs_t)
            want[sl] = oracle.retrieve(ref, pl)
            total += pl.bytes
        assert np.array_equal(out.view(bits), want.view(bits)), (kind, val)
        assert rinfo["bytes_total"] == total
        err = out.astype(np.float64) - x
        if kind == "rel":
            assert np.abs(err).max() <= val * rng
        else:
            assert 20 * math.log10(rng / math.sqrt(np.mean(err ** 2))) >= val
    bs.close()
