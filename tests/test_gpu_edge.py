"""GPU edge cases against the oracle: streams without planes (B = 0) in a
group whose step is not zero, all-zero fields, and retrieval state handed
out dirty by the device memory pool.

A field that varies only along axis 0 makes every decomposition stream of
level-0 regions 0 and 1 (and S2, S3 of region 2) all zero while their group,
level 0, has a nonzero maximum: those streams have no planes and are never
decoded, so their code buffers hold whatever the pool handed out.  Each case
first refactors and fully retrieves a random field of the same shape and
frees it, so that the buffers the next handle gets back hold nonzero codes."""
import numpy as np
import pytest

import fieldgen
import oracle

from test_gpu_parity import _bits, _check_metadata, _check_retrievals, _check_streams, _schemes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _apc():
    import paper_2609_04573_amd as apc
    return apc


def _dirty_pool(shape, gs):
    apc = _apc()
    noise = np.random.default_rng(99).standard_normal(shape).astype(np.float32)
    h = apc.refactor(torch.from_numpy(noise).cuda(), gs)
    full = [h.stream_info(s)["B"] for s in range(h.num_streams)]
    h.retrieve_planes(full)
    h.retrieve(apc.Target("rel", 1e-6))
    torch.cuda.synchronize()
    h.close()


def _axis0_field(shape, seed=3):
    rng = np.random.default_rng(seed)
    prof = rng.standard_normal((shape[0],) + (1,) * (len(shape) - 1))
    return np.ascontiguousarray(np.broadcast_to(prof, shape)).astype(np.float32)


@pytest.mark.parametrize("scheme", [("level", 3, None, 0), ("region", 3, (2, 1, 0), 0), ("level", 1, None, 1)],
                         ids=str)
def test_axis0_only_field_streams_without_planes(scheme):
    apc = _apc()
    shape = (24, 20, 33)
    x = _axis0_field(shape)
    gs, os_ = _schemes(*scheme)
    ref = oracle.refactor(x, os_)
    assert any(st.meta.B == 0 and ref.groups[st.group].delta > 0 for st in ref.streams)
    _dirty_pool(shape, gs)
    h = apc.refactor(torch.from_numpy(x).cuda(), gs)
    _check_metadata(h, ref)
    _check_streams(h, ref)
    _check_retrievals(h, ref, x)
    full = [st.meta.B for st in ref.streams]
    got = h.retrieve_planes(full).cpu().numpy()
    assert np.array_equal(_bits(got), _bits(oracle.pipeline.quantized_field(ref)))
    h.close()


@pytest.mark.parametrize("shape", [(24, 20, 33), (64, 64, 64), (1800, 360)], ids=str)
def test_all_zero_field(shape):
    apc = _apc()
    x = np.zeros(shape, np.float32)
    scheme = ("level", 3, None, 0)
    gs, os_ = _schemes(*scheme)
    ref = oracle.refactor(x, os_)
    _dirty_pool(shape, gs)
    h = apc.refactor(torch.from_numpy(x).cuda(), gs)
    _check_metadata(h, ref)
    _check_streams(h, ref)
    for val in (1e-3, 1e-9):
        out, info = h.retrieve(apc.Target("abs", val))
        got = out.cpu().numpy()
        pl = oracle.plan(ref, oracle.Target("abs", val))
        assert np.array_equal(_bits(got), _bits(oracle.retrieve(ref, pl)))
        assert not np.signbit(got).any()  # +0.0 everywhere, as the oracle
    h.close()


def test_bump_field_after_dirty_pool_float64():
    """float64 codes (int64) with a dirty pool: a smooth field where some
    decomposition streams are zero only at the finest lifting level."""
    apc = _apc()
    shape = (17, 30, 45)
    x = fieldgen.polynomial_field(shape, [[0, 3], [0, 0, 1], [2]], dtype=np.float64)
    gs, os_ = _schemes("level", 3, None, 1)
    ref = oracle.refactor(x, os_)
    noise = np.random.default_rng(98).standard_normal(shape)
    h0 = apc.refactor(torch.from_numpy(noise).cuda(), gs)
    h0.retrieve_planes([h0.stream_info(s)["B"] for s in range(h0.num_streams)])
    torch.cuda.synchronize()
    h0.close()
    h = apc.refactor(torch.from_numpy(x).cuda(), gs)
    _check_metadata(h, ref)
    _check_streams(h, ref)
    for rel in (1e-3, 1e-8):
        pl = oracle.plan(ref, oracle.Target("rel", rel))
        out, _ = h.retrieve(apc.Target("rel", rel))
        assert np.array_equal(_bits(out.cpu().numpy()), _bits(oracle.retrieve(ref, pl)))
    h.close()
