"""The library's interpreters (greedy, dynamic program, best-first search,
the paper's choice) against the oracle's, on the CPU: a planning-only handle
is rebuilt from bytes the oracle's refactoring fills in
(apc_deserialize_host), so no device is needed; plans must match plane for
plane, with the same bound, bytes and step count."""
import numpy as np
import pytest

import fieldgen
import oracle
from oracle import interp
from oracle.pipeline import target_tau

from test_serialize import oracle_bytes

TARGETS = [("rel", 1e-2), ("rel", 1e-4), ("rel", 1e-6), ("psnr", 40), ("psnr", 80)]
ORACLE = {"dp": interp.dp_plan, "best_first": interp.best_first_plan, "paper": interp.paper_plan}


def _apc():
    import paper_2609_04573_amd as apc
    return apc


@pytest.mark.parametrize("scheme", [oracle.Scheme(kind="level", cd_axis=0), oracle.Scheme(kind="region"),
                                    oracle.Scheme(kind="region", order=(0, 2, 1), cd_axis=1),
                                    oracle.Scheme(kind="level"),
                                    oracle.Scheme(kind="region", encoding="negabinary_xor", lossless=True),
                                    oracle.Scheme(kind="level", cd_axis=0, encoding="negabinary")], ids=str)
def test_library_plans_equal_the_oracle(config1_field, scheme):
    apc = _apc()
    ref = oracle.refactor(config1_field, scheme)
    h = apc.deserialize_host(oracle_bytes(ref))
    for name in ("greedy", "dp", "best_first", "paper"):
        h.set_interpreter(name)
        for kind, val in TARGETS:
            planes, info = h.plan(apc.Target(kind, val))
            tau, mode = target_tau(ref, oracle.Target(kind, val))
            pl = oracle.plan(ref, oracle.Target(kind, val)) if name == "greedy" else ORACLE[name](ref, tau, mode)
            assert planes == pl.planes, (name, kind, val)
            assert info["bound"] == pl.bound and info["bytes_total"] == pl.bytes and info["nsteps"] == pl.nsteps
            assert info["bound"] <= tau
    h.close()


def test_interpreters_fetch_fewer_bytes_than_greedy_on_a_turbulent_field():
    apc = _apc()
    x = fieldgen.power_law_field((40, 48, 56), seed=9)
    ref = oracle.refactor(x, oracle.Scheme(kind="level", cd_axis=0))
    h = apc.deserialize_host(oracle_bytes(ref))
    saved = 0
    for kind, val in TARGETS:
        _, g = h.plan(apc.Target(kind, val))
        h.set_interpreter("paper")
        _, p = h.plan(apc.Target(kind, val))
        h.set_interpreter("greedy")
        assert p["bytes_total"] <= g["bytes_total"]
        saved += g["bytes_total"] - p["bytes_total"]
    assert saved > 0
    h.close()


def test_host_only_handle_refuses_device_work(config1_field):
    apc = _apc()
    ref = oracle.refactor(config1_field, oracle.Scheme(kind="region"))
    h = apc.deserialize_host(oracle_bytes(ref))
    assert h.num_streams == len(ref.streams) and h.metadata()["L"] == ref.L
    with pytest.raises(apc.ApcError) as ei:
        h.stream_blob(0)
    assert ei.value.status == -1 and "no device data" in str(ei.value)
    with pytest.raises(apc.ApcError):
        apc.apc._check(apc.apc.library().apc_set_interpreter(h._h, 9))
    # batched retrieval refuses it before touching any output (the output
    # pointer below is never dereferenced), and refuses null arguments
    import ctypes
    lib = apc.apc.library()
    hs = (ctypes.c_void_p * 1)(h._h)
    tg = (apc.apc._Target * 1)(apc.Target("rel", 1e-3)._c())
    outs = (ctypes.c_void_p * 1)(16)
    assert lib.apc_retrieve_batch(hs, 1, tg, outs, None, None) == -1
    assert lib.apc_retrieve_batch(None, 1, tg, outs, None, None) == -1
    assert lib.apc_retrieve_batch(hs, 0, tg, outs, None, None) == -1
    h.close()
