"""GPU tests of the continuous-batching retrieval server: every result in a
concurrent mix equals the same request made alone and the oracle's
reconstruction for its plan (bit for bit), several requests are on the
device at once (merged into batches), only missing planes are fetched, and
admission respects the HBM budget."""
import numpy as np
import pytest

import fieldgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EB = (1e-2, 1e-3, 1e-4, 1e-5, 1e-6)
PSNR = (40, 50, 60, 70, 80, 90, 100)


def _apc():
    import paper_2609_04573_amd as apc
    return apc


def _setup(n=96, nf=4):
    apc = _apc()
    xs = [torch.from_numpy(fieldgen.power_law_field((n, n, n), seed=3 + i)).cuda() for i in range(nf)]
    schemes = [apc.Scheme(kind="level", cd_axis=0), apc.Scheme(kind="region"),
               apc.Scheme(kind="level"), apc.Scheme(kind="region", order=(0, 1, 2), cd_axis=2)][:nf]
    return xs, schemes


def _requests(nreq, nf, seed):
    apc = _apc()
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(nreq):
        f = int(rng.integers(0, nf))
        if rng.random() < 0.5:
            reqs.append((f, apc.Target("rel", float(rng.choice(EB)))))
        else:
            reqs.append((f, apc.Target("psnr", float(rng.choice(PSNR)))))
    return reqs


def _oracle_refs(xs, schemes):
    refs = []
    for x, s in zip(xs, schemes):
        refs.append(oracle.refactor(x.cpu().numpy(), oracle.Scheme(kind=s.kind, degree=s.degree, order=s.order,
                                                                    cd_axis=s.cd_axis)))
    return refs


@pytest.mark.timeout(600)
def test_server_mix_equals_alone():
    apc = _apc()
    xs, schemes = _setup()
    served = apc.refactor_batch(xs, schemes)
    srv = apc.Server(served, budget_bytes=4 << 30, max_slots=4, max_batch=8)
    reqs = _requests(80, len(xs), seed=100)
    outs = [torch.empty_like(xs[f]) for f, _ in reqs]
    tickets = [srv.submit(f, t, o) for (f, t), o in zip(reqs, outs)]
    infos = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs)
    assert st["max_running"] >= 2, st
    alone = [apc.refactor(x, s) for x, s in zip(xs, schemes)]
    fetched = sum(i["bytes_fetched"] for i in infos)
    total = sum(i["bytes_total"] for i in infos)
    assert fetched < total  # later requests reuse planes fetched by earlier ones
    refs = _oracle_refs(xs, schemes)
    for k, ((f, t), o) in enumerate(zip(reqs, outs)):
        want, _ = alone[f].retrieve(t)
        assert torch.equal(o.view(torch.int32), want.view(torch.int32)), (k, f, t)
        pl = oracle.plan(refs[f], oracle.Target(t.kind, t.value))
        assert infos[k]["bytes_total"] == pl.bytes
        ow = oracle.retrieve(refs[f], pl)
        assert np.array_equal(o.cpu().numpy().view(np.uint32), ow.view(np.uint32)), (k, f, t)
    for h in alone + served:
        h.close()


def test_server_batches_requests_submitted_together():
    """Requests queued while a batch runs join the next batch: with one slot,
    a burst of submissions is served in merged batches (several requests on
    the device at once) and every output still equals the oracle's."""
    apc = _apc()
    xs, schemes = _setup(n=64, nf=4)
    served = apc.refactor_batch(xs, schemes)
    srv = apc.Server(served, budget_bytes=4 << 30, max_slots=1, max_batch=16)
    reqs = _requests(40, len(xs), seed=11)
    outs = [torch.empty_like(xs[f]) for f, _ in reqs]
    tickets = [srv.submit(f, t, o) for (f, t), o in zip(reqs, outs)]
    for tk in tickets:
        srv.wait(tk)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["max_running"] >= 2, st
    refs = _oracle_refs(xs, schemes)
    for (f, t), o in zip(reqs, outs):
        ow = oracle.retrieve(refs[f], oracle.plan(refs[f], oracle.Target(t.kind, t.value)))
        assert np.array_equal(o.cpu().numpy().view(np.uint32), ow.view(np.uint32)), (f, t)
    for h in served:
        h.close()


def test_server_one_slot_serializes_and_matches():
    apc = _apc()
    xs, schemes = _setup(n=64, nf=2)
    served = apc.refactor_batch(xs, schemes)
    srv = apc.Server(served, budget_bytes=4 << 30, max_slots=1, max_batch=1)
    reqs = _requests(20, len(xs), seed=7)
    outs = [torch.empty_like(xs[f]) for f, _ in reqs]
    tickets = [srv.submit(f, t, o) for (f, t), o in zip(reqs, outs)]
    for t in tickets:
        srv.wait(t)
    assert srv.stats()["max_running"] == 1
    srv.close()
    alone = [apc.refactor(x, s) for x, s in zip(xs, schemes)]
    for (f, t), o in zip(reqs, outs):
        want, _ = alone[f].retrieve(t)
        assert torch.equal(o.view(torch.int32), want.view(torch.int32))
    for h in alone + served:
        h.close()


def test_server_refuses_requests_over_budget_and_below_floor():
    apc = _apc()
    xs, schemes = _setup(n=32, nf=1)
    hs = apc.refactor_batch(xs, schemes)
    srv = apc.Server(hs, budget_bytes=1024, max_slots=2)
    with pytest.raises(apc.ApcError) as ei:
        srv.submit(0, apc.Target("rel", 1e-3), torch.empty_like(xs[0]))
    assert ei.value.status == -7
    srv.close()
    c = torch.full((16, 16, 16), 1.5, device="cuda")
    hc = apc.refactor(c, apc.Scheme())
    srv2 = apc.Server([hc], budget_bytes=1 << 30, max_slots=2)
    with pytest.raises(apc.BelowFloor):
        srv2.submit(0, apc.Target("rel", 1e-3), torch.empty_like(c))
    o = torch.empty_like(c)
    srv2.wait(srv2.submit(0, apc.Target("abs", 1e-3), o))
    assert torch.equal(o, c)
    srv2.close()
    hc.close()
    for h in hs:
        h.close()
