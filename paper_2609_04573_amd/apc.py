"""ctypes binding of ``libapc.so`` (argument marshalling only).

Every step of refactoring and retrieval runs in the library's HIP kernels;
PyTorch only provides device memory and the current HIP stream.  There is no
fallback: if the library is not built this module raises on import.
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")

# torch first: its bundled HIP runtime is then the one the library binds to
# (both carry the soname libamdhip64.so.7), so device memory and streams
# from torch and the library's own calls share one runtime instance
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

APC_OK = 0
APC_E_INVALID = -1
APC_E_DTYPE = -2
APC_E_NONFINITE = -3
APC_E_BELOW_FLOOR = -4
APC_E_OOM = -5
APC_E_HIP = -6
APC_E_BUSY = -7
APC_E_CORRUPT = -8
APC_E_NODEVICE = -9

APC_F32, APC_F64 = 0, 1
PER_LEVEL, PER_REGION = 0, 1
TARGET_KINDS = {"abs": 0, "rel": 1, "psnr": 2, "rmse": 3}
MODES = {"eb": 0, "psnr": 1}

EXPORTED = [
    "apc_refactor", "apc_plan", "apc_retrieve", "apc_retrieve_planes", "apc_retrieve_batch", "apc_select_pipeline", "apc_free",
    "apc_strerror", "apc_last_error", "apc_num_streams", "apc_num_groups", "apc_num_points", "apc_stream_info",
    "apc_stream_blob", "apc_metadata_json", "apc_axis_norms", "apc_profile_enable", "apc_profile_report",
    "apc_refactor_batch", "apc_ladder_create", "apc_ladder_launch", "apc_ladder_free", "apc_server_create",
    "apc_server_submit", "apc_server_poll", "apc_server_wait", "apc_server_stats", "apc_server_reset_stats",
    "apc_server_destroy", "apc_tune_tiles", "apc_tile_override", "apc_tile_width", "apc_profile_only",
    "apc_retrieve_static", "apc_field_info", "apc_serialize", "apc_deserialize", "apc_deserialize_host",
    "apc_set_interpreter", "apc_blocks_refactor", "apc_blocks_retrieve", "apc_blocks_set_interpreter",
    "apc_blocks_info", "apc_blocks_blob", "apc_blocks_free",
]
INTERPRETERS = {"greedy": 0, "dp": 1, "best_first": 2, "paper": 3}
ENCODINGS = {"generic": 0, "negabinary": 1, "negabinary_xor": 2}


class _Scheme(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("degree", ctypes.c_int32), ("order", ctypes.c_int32 * 3),
                ("cd_axis", ctypes.c_int32), ("levels", ctypes.c_int32), ("lossless", ctypes.c_int32),
                ("encoding", ctypes.c_int32)]


class _Target(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("value", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("bytes_total", ctypes.c_int64), ("bytes_fetched", ctypes.c_int64), ("bound", ctypes.c_double),
                ("tau", ctypes.c_double), ("bitrate", ctypes.c_double), ("n_streams", ctypes.c_int32),
                ("nsteps", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_lib.apc_refactor.argtypes = [_vp, _i32, ctypes.POINTER(_i64), _i32, ctypes.POINTER(_Scheme), _vp, ctypes.POINTER(_vp)]
_lib.apc_plan.argtypes = [_vp, ctypes.POINTER(_Target), ctypes.POINTER(_i32), ctypes.POINTER(_Info)]
_lib.apc_retrieve.argtypes = [_vp, ctypes.POINTER(_Target), _vp, ctypes.POINTER(_Info), _vp]
_lib.apc_retrieve_planes.argtypes = [_vp, ctypes.POINTER(_i32), _vp, _vp]
_lib.apc_retrieve_batch.argtypes = [ctypes.POINTER(_vp), _i32, ctypes.POINTER(_Target), ctypes.POINTER(_vp),
                                    ctypes.POINTER(_Info), _vp]
_lib.apc_retrieve_static.argtypes = [_vp, ctypes.POINTER(_Target), _vp, ctypes.POINTER(_Info), _vp]
_lib.apc_field_info.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
_lib.apc_serialize.argtypes = [_vp, _vp, _i64, ctypes.POINTER(_i64)]
_lib.apc_deserialize.argtypes = [ctypes.c_char_p, _i64, _vp, ctypes.POINTER(_vp)]
_lib.apc_deserialize_host.argtypes = [ctypes.c_char_p, _i64, ctypes.POINTER(_vp)]
_lib.apc_set_interpreter.argtypes = [_vp, _i32]
_lib.apc_blocks_refactor.argtypes = [_vp, _i32, ctypes.POINTER(_i64), _i32, ctypes.POINTER(_i64),
                                     ctypes.POINTER(_Scheme), _i64, _vp, ctypes.POINTER(_vp)]
_lib.apc_blocks_retrieve.argtypes = [_vp, ctypes.POINTER(_Target), _vp, ctypes.POINTER(_Info), _vp]
_lib.apc_blocks_set_interpreter.argtypes = [_vp, _i32]
_lib.apc_blocks_info.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]
_lib.apc_blocks_blob.argtypes = [_vp, _i64, ctypes.POINTER(_vp), ctypes.POINTER(_i64)]
_lib.apc_blocks_free.argtypes = [_vp]
_lib.apc_blocks_free.restype = None
_lib.apc_select_pipeline.argtypes = [_vp, _i32, ctypes.POINTER(_i64), _i32, _i32, ctypes.POINTER(_Scheme), _vp]
_lib.apc_free.argtypes = [_vp]
_lib.apc_free.restype = None
_lib.apc_strerror.argtypes = [_i32]
_lib.apc_strerror.restype = ctypes.c_char_p
_lib.apc_last_error.restype = ctypes.c_char_p
_lib.apc_num_streams.argtypes = [_vp]
_lib.apc_num_groups.argtypes = [_vp]
_lib.apc_num_points.argtypes = [_vp]
_lib.apc_num_points.restype = _i64
_lib.apc_stream_info.argtypes = [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i32), ctypes.POINTER(_i64),
                                 ctypes.POINTER(_i64)]
_lib.apc_stream_blob.argtypes = [_vp, _i32, _vp, _i64]
_lib.apc_metadata_json.argtypes = [_vp, ctypes.c_char_p, _i64, ctypes.POINTER(_i64)]
_lib.apc_axis_norms.argtypes = [_i64, _i32, _i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.apc_profile_enable.argtypes = [_i32]
_lib.apc_refactor_batch.argtypes = [ctypes.POINTER(_vp), _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i32),
                                    ctypes.POINTER(_Scheme), _i32, _vp, ctypes.POINTER(_vp)]
_lib.apc_ladder_create.argtypes = [_vp, ctypes.POINTER(_Target), _i32, ctypes.POINTER(_vp), _vp,
                                   ctypes.POINTER(_vp)]
_lib.apc_ladder_launch.argtypes = [_vp, _vp]
_lib.apc_ladder_free.argtypes = [_vp]
_lib.apc_ladder_free.restype = None
_lib.apc_server_create.argtypes = [ctypes.POINTER(_vp), _i32, _i64, _i32, _i32, ctypes.POINTER(_vp)]
_lib.apc_server_submit.argtypes = [_vp, _i32, ctypes.POINTER(_Target), _vp, ctypes.POINTER(_i64)]
_lib.apc_server_poll.argtypes = [_vp, _i64, ctypes.POINTER(_i32)]
_lib.apc_server_wait.argtypes = [_vp, _i64, ctypes.POINTER(_Info)]
_lib.apc_server_stats.argtypes = [_vp] + [ctypes.POINTER(ctypes.c_double)] * 3 + [ctypes.POINTER(_i64)] * 2
_lib.apc_server_reset_stats.argtypes = [_vp]
_lib.apc_server_destroy.argtypes = [_vp]
_lib.apc_server_destroy.restype = None
_lib.apc_profile_report.argtypes = [ctypes.c_char_p, _i64, ctypes.POINTER(_i64)]
_lib.apc_tune_tiles.argtypes = [_vp, _i32, ctypes.POINTER(_i64), _i32, _i32, _vp, ctypes.POINTER(_i32),
                                ctypes.POINTER(ctypes.c_double)]
_lib.apc_tile_override.argtypes = [_i32]
_lib.apc_profile_only.argtypes = [ctypes.c_char_p]
_lib.apc_tile_width.argtypes = [_i32, _i64, _i64, ctypes.POINTER(_i32)]
for _name in ("apc_refactor", "apc_plan", "apc_retrieve", "apc_retrieve_planes", "apc_select_pipeline",
              "apc_stream_info", "apc_stream_blob", "apc_metadata_json", "apc_axis_norms", "apc_profile_enable",
              "apc_profile_report", "apc_refactor_batch", "apc_ladder_create", "apc_ladder_launch",
              "apc_server_create", "apc_server_submit", "apc_server_poll", "apc_server_wait", "apc_server_stats",
              "apc_server_reset_stats", "apc_tune_tiles", "apc_tile_override", "apc_tile_width",
              "apc_profile_only", "apc_retrieve_static", "apc_field_info", "apc_serialize", "apc_deserialize",
              "apc_deserialize_host", "apc_set_interpreter", "apc_blocks_refactor", "apc_blocks_retrieve",
              "apc_blocks_set_interpreter", "apc_blocks_info", "apc_blocks_blob"):
    getattr(_lib, _name).restype = _i32


class ApcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_lib.apc_strerror(status).decode()} ({status}): {msg}")
        self.status = status


class BelowFloor(ApcError):
    pass


def _check(status: int):
    if status != APC_OK:
        msg = (_lib.apc_last_error() or b"").decode(errors="replace")
        if status == APC_E_BELOW_FLOOR:
            raise BelowFloor(status, msg)
        raise ApcError(status, msg)


@dataclass(frozen=True)
class Scheme:
    kind: str = "level"                      # "level", "region", or (refactor only) "auto" / "auto_psnr"
    degree: int = 3
    order: Optional[Tuple[int, ...]] = None  # per-region pass order (axes)
    cd_axis: Optional[int] = None
    levels: int = 0
    lossless: bool = False                   # zero-word suppression of stored planes
    encoding: str = "generic"                # "generic", "negabinary" or "negabinary_xor"

    def _c(self, ndim: int) -> _Scheme:
        s = _Scheme()
        s.kind = {"level": PER_LEVEL, "region": PER_REGION, "auto": 2, "auto_psnr": 3}[self.kind]
        s.degree = self.degree
        order = self.order if self.order is not None else tuple(range(ndim - 1, -1, -1))
        for i in range(3):
            s.order[i] = order[i] if i < len(order) else 0
        s.cd_axis = -1 if self.cd_axis is None else int(self.cd_axis)
        s.levels = int(self.levels or 0)
        s.lossless = 1 if self.lossless else 0
        s.encoding = ENCODINGS[self.encoding]
        return s

    @staticmethod
    def _from_c(s: _Scheme, ndim: int) -> "Scheme":
        return Scheme(kind="level" if s.kind == PER_LEVEL else "region", degree=s.degree,
                      order=None if s.kind == PER_LEVEL else tuple(s.order[i] for i in range(ndim)),
                      cd_axis=None if s.cd_axis < 0 else s.cd_axis, levels=s.levels, lossless=bool(s.lossless),
                      encoding={v: k for k, v in ENCODINGS.items()}[s.encoding])


@dataclass(frozen=True)
class Target:
    kind: str     # "abs", "rel", "psnr", "rmse"
    value: float

    def _c(self) -> _Target:
        t = _Target()
        t.kind = TARGET_KINDS[self.kind]
        t.value = float(self.value)
        return t


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return APC_F32
    if t.dtype == torch.float64:
        return APC_F64
    raise ApcError(APC_E_DTYPE, f"unsupported dtype {t.dtype}")


def _info_dict(inf: _Info) -> dict:
    return {k: getattr(inf, k) for k, _ in _Info._fields_}


class Handle:
    """A refactored field (owns device plane streams; not thread-safe)."""

    def __init__(self, ptr: int, shape: Tuple[int, ...], dtype):
        self._h = ctypes.c_void_p(ptr)
        self.shape = tuple(shape)
        self.dtype = dtype

    def close(self):
        if self._h:
            _lib.apc_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_streams(self) -> int:
        return _lib.apc_num_streams(self._h)

    def plan(self, target: Target):
        planes = (ctypes.c_int32 * self.num_streams)()
        inf = _Info()
        _check(_lib.apc_plan(self._h, ctypes.byref(target._c()), planes, ctypes.byref(inf)))
        return list(planes), _info_dict(inf)

    def retrieve(self, target: Target, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, device="cuda")
        assert out.is_contiguous() and out.dtype == self.dtype and tuple(out.shape) == self.shape
        inf = _Info()
        _check(_lib.apc_retrieve(self._h, ctypes.byref(target._c()), ctypes.c_void_p(out.data_ptr()),
                                 ctypes.byref(inf), _stream_ptr(stream)))
        return out, _info_dict(inf)

    def retrieve_static(self, target: Target, out=None, stream=None):
        """apc_retrieve_static: the same output as retrieve(), decoded from no
        resident planes into the library's static device scratch (no device
        allocation by the library)."""
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, device="cuda")
        assert out.is_contiguous() and out.dtype == self.dtype and tuple(out.shape) == self.shape
        inf = _Info()
        _check(_lib.apc_retrieve_static(self._h, ctypes.byref(target._c()), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.byref(inf), _stream_ptr(stream)))
        return out, _info_dict(inf)

    def retrieve_planes(self, planes: Sequence[int], out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, device="cuda")
        assert out.is_contiguous() and out.dtype == self.dtype and tuple(out.shape) == self.shape
        arr = (ctypes.c_int32 * self.num_streams)(*[int(p) for p in planes])
        _check(_lib.apc_retrieve_planes(self._h, arr, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def stream_info(self, s: int) -> dict:
        n, B, mx, nb = _i64(), _i32(), _i64(), _i64()
        _check(_lib.apc_stream_info(self._h, s, ctypes.byref(n), ctypes.byref(B), ctypes.byref(mx), ctypes.byref(nb)))
        return {"n": n.value, "B": B.value, "maxabs": mx.value, "blob_bytes": nb.value}

    def stream_blob(self, s: int) -> bytes:
        nb = self.stream_info(s)["blob_bytes"]
        buf = ctypes.create_string_buffer(max(1, nb))
        _check(_lib.apc_stream_blob(self._h, s, buf, max(1, nb)))
        return buf.raw[:nb]

    def set_interpreter(self, name: str) -> None:
        """Retrieval interpreter: "greedy" (default), "dp", "best_first" or
        "paper" (dp for per-region, best_first for per-level)."""
        _check(_lib.apc_set_interpreter(self._h, INTERPRETERS[name]))

    def serialize(self) -> bytes:
        """The stored representation as bytes (apc_serialize)."""
        ln = _i64()
        _check(_lib.apc_serialize(self._h, None, 0, ctypes.byref(ln)))
        buf = ctypes.create_string_buffer(max(1, ln.value))
        _check(_lib.apc_serialize(self._h, buf, ln.value, ctypes.byref(ln)))
        return buf.raw[:ln.value]

    @property
    def scheme(self) -> "Scheme":
        """The scheme the field was refactored with (the chosen one for
        "auto" kinds)."""
        c = self.metadata()["scheme"]
        d = len(self.shape)
        return Scheme(kind="level" if c["kind"] == PER_LEVEL else "region", degree=c["degree"],
                      order=None if c["kind"] == PER_LEVEL else tuple(c["order"][:d]),
                      cd_axis=None if c["cd_axis"] < 0 else c["cd_axis"], levels=c["levels"],
                      lossless=bool(c["lossless"]), encoding={v: k for k, v in ENCODINGS.items()}[c["encoding"]])

    def metadata(self) -> dict:
        ln = _i64()
        _check(_lib.apc_metadata_json(self._h, None, 0, ctypes.byref(ln)))
        buf = ctypes.create_string_buffer(ln.value + 1)
        _check(_lib.apc_metadata_json(self._h, buf, ln.value + 1, None))
        return json.loads(buf.value.decode())


def refactor(field, scheme: Scheme = Scheme(), stream=None) -> Handle:
    """Refactor a contiguous CUDA (HIP) float32/float64 tensor of 1-3 dims."""
    assert field.is_cuda and field.is_contiguous(), "field must be a contiguous device tensor"
    dims = (ctypes.c_int64 * field.dim())(*field.shape)
    out = ctypes.c_void_p()
    _check(_lib.apc_refactor(ctypes.c_void_p(field.data_ptr()), _dtype_code(field), dims, field.dim(),
                             ctypes.byref(scheme._c(field.dim())), _stream_ptr(stream), ctypes.byref(out)))
    return Handle(out.value, tuple(field.shape), field.dtype)


def check_serialized(data: bytes) -> None:
    """Check serialized bytes without a device (raises ApcError, status
    APC_E_CORRUPT, naming the first failed check)."""
    _check(_lib.apc_deserialize(data, len(data), None, None))


def deserialize(data: bytes, stream=None) -> Handle:
    """A handle from apc_serialize bytes (streams uploaded on the stream)."""
    import torch
    out = ctypes.c_void_p()
    _check(_lib.apc_deserialize(data, len(data), _stream_ptr(stream), ctypes.byref(out)))
    dims = (ctypes.c_int64 * 3)()
    nd, dt = _i32(), _i32()
    _check(_lib.apc_field_info(out, dims, ctypes.byref(nd), ctypes.byref(dt)))
    return Handle(out.value, tuple(dims[i] for i in range(nd.value)),
                  torch.float32 if dt.value == APC_F32 else torch.float64)


def deserialize_host(data: bytes) -> Handle:
    """A planning-only handle from apc_serialize bytes (no device needed)."""
    out = ctypes.c_void_p()
    _check(_lib.apc_deserialize_host(data, len(data), ctypes.byref(out)))
    dims = (ctypes.c_int64 * 3)()
    nd, dt = _i32(), _i32()
    _check(_lib.apc_field_info(out, dims, ctypes.byref(nd), ctypes.byref(dt)))
    return Handle(out.value, tuple(dims[i] for i in range(nd.value)), None)


def retrieve_batch(handles, targets, outs=None, stream=None):
    """Retrieve many handles (one dtype; a handle may repeat) in shared
    launches; returns (outputs, infos), each output equal to that request's
    retrieve() alone."""
    import torch
    n = len(handles)
    assert n == len(targets) and n > 0
    if outs is None:
        outs = [torch.empty(h.shape, dtype=h.dtype, device="cuda") for h in handles]
    for h, o in zip(handles, outs):
        assert o.is_contiguous() and o.dtype == h.dtype and tuple(o.shape) == h.shape
    hs = (_vp * n)(*[h._h for h in handles])
    tg = (_Target * n)(*[t._c() for t in targets])
    ptrs = (_vp * n)(*[o.data_ptr() for o in outs])
    infs = (_Info * n)()
    _check(_lib.apc_retrieve_batch(hs, n, tg, ptrs, infs, _stream_ptr(stream)))
    return outs, [_info_dict(i) for i in infs]


def refactor_batch(fields, schemes, stream=None) -> List[Handle]:
    """Refactor many contiguous device tensors (one dtype) in shared launches."""
    nf = len(fields)
    assert nf == len(schemes) and nf > 0
    dt = _dtype_code(fields[0])
    ptrs = (ctypes.c_void_p * nf)(*[f.data_ptr() for f in fields])
    dims = []
    for f in fields:
        assert f.is_cuda and f.is_contiguous() and _dtype_code(f) == dt
        dims.extend(int(v) for v in f.shape)
    cdims = (ctypes.c_int64 * len(dims))(*dims)
    nds = (ctypes.c_int32 * nf)(*[f.dim() for f in fields])
    cs = (_Scheme * nf)(*[sc._c(f.dim()) for sc, f in zip(schemes, fields)])
    outs = (ctypes.c_void_p * nf)()
    _check(_lib.apc_refactor_batch(ptrs, dt, cdims, nds, cs, nf, _stream_ptr(stream), outs))
    return [Handle(outs[i], tuple(f.shape), f.dtype) for i, f in enumerate(fields)]


class Ladder:
    """A retrieval ladder captured as one HIP graph (replayable)."""

    def __init__(self, handle: Handle, targets: Sequence[Target], outs=None, stream=None):
        import torch
        n = len(targets)
        self.handle = handle
        self.outs = outs if outs is not None else [torch.empty(handle.shape, dtype=handle.dtype, device="cuda")
                                                   for _ in range(n)]
        tg = (_Target * n)(*[t._c() for t in targets])
        ptrs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in self.outs])
        out = ctypes.c_void_p()
        _check(_lib.apc_ladder_create(handle._h, tg, n, ptrs, _stream_ptr(stream), ctypes.byref(out)))
        self._p = out

    def launch(self, stream=None):
        _check(_lib.apc_ladder_launch(self._p, _stream_ptr(stream)))
        return self.outs

    def close(self):
        if self._p:
            _lib.apc_ladder_free(self._p)
            self._p = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching retrieval server over resident refactored fields."""

    def __init__(self, handles: Sequence[Handle], budget_bytes: int, max_slots: int = 4, max_batch: int = 16):
        """max_slots batches in flight, up to max_batch requests per batch
        (max_slots = max_batch = 1: one request at a time)."""
        self.handles = list(handles)
        arr = (ctypes.c_void_p * len(self.handles))(*[h._h.value for h in self.handles])
        out = ctypes.c_void_p()
        _check(_lib.apc_server_create(arr, len(self.handles), int(budget_bytes), int(max_slots), int(max_batch),
                                      ctypes.byref(out)))
        self._p = out

    def submit(self, field: int, target: Target, out) -> int:
        h = self.handles[field]
        assert out.is_contiguous() and out.dtype == h.dtype and tuple(out.shape) == h.shape
        t = _i64()
        _check(_lib.apc_server_submit(self._p, int(field), ctypes.byref(target._c()), ctypes.c_void_p(out.data_ptr()),
                                      ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> bool:
        d = _i32()
        _check(_lib.apc_server_poll(self._p, int(ticket), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int) -> dict:
        inf = _Info()
        _check(_lib.apc_server_wait(self._p, int(ticket), ctypes.byref(inf)))
        return _info_dict(inf)

    def stats(self) -> dict:
        p50, p99, mean = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        done, mr = _i64(), _i64()
        _check(_lib.apc_server_stats(self._p, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(mean),
                                     ctypes.byref(done), ctypes.byref(mr)))
        return {"p50_ms": p50.value, "p99_ms": p99.value, "mean_ms": mean.value, "completed": done.value,
                "max_running": mr.value}

    def reset_stats(self):
        _check(_lib.apc_server_reset_stats(self._p))

    def close(self):
        if self._p:
            _lib.apc_server_destroy(self._p)
            self._p = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BlockSet:
    """A host-resident field refactored block by block (out of core): the
    representation stays in host memory; retrievals upload only the planned
    planes of each block."""

    def __init__(self, field_host, block, scheme: Scheme = Scheme(), group_bytes: int = 4 << 30, stream=None):
        import numpy as np
        a = np.ascontiguousarray(field_host)
        if a.dtype == np.float32:
            dt = APC_F32
        elif a.dtype == np.float64:
            dt = APC_F64
        else:
            raise ApcError(APC_E_DTYPE, f"unsupported dtype {a.dtype}")
        self.shape, self.dtype = a.shape, a.dtype
        dims = (ctypes.c_int64 * a.ndim)(*a.shape)
        blk = (ctypes.c_int64 * a.ndim)(*[int(b) for b in block])
        out = ctypes.c_void_p()
        _check(_lib.apc_blocks_refactor(ctypes.c_void_p(a.ctypes.data), dt, dims, a.ndim, blk,
                                        ctypes.byref(scheme._c(a.ndim)), int(group_bytes), _stream_ptr(stream),
                                        ctypes.byref(out)))
        self._p = out

    def info(self) -> dict:
        nb, sb = _i64(), _i64()
        lo, hi = ctypes.c_double(), ctypes.c_double()
        _check(_lib.apc_blocks_info(self._p, ctypes.byref(nb), ctypes.byref(sb), ctypes.byref(lo), ctypes.byref(hi)))
        return {"blocks": nb.value, "stored_bytes": sb.value, "xmin": lo.value, "xmax": hi.value}

    def blob(self, b: int) -> bytes:
        p, n = ctypes.c_void_p(), _i64()
        _check(_lib.apc_blocks_blob(self._p, int(b), ctypes.byref(p), ctypes.byref(n)))
        return ctypes.string_at(p, n.value)

    def set_interpreter(self, name: str) -> None:
        _check(_lib.apc_blocks_set_interpreter(self._p, INTERPRETERS[name]))

    def retrieve(self, target: Target, out=None, stream=None):
        import numpy as np
        if out is None:
            out = np.empty(self.shape, dtype=self.dtype)
        assert out.flags.c_contiguous and out.dtype == self.dtype and out.shape == self.shape
        inf = _Info()
        _check(_lib.apc_blocks_retrieve(self._p, ctypes.byref(target._c()), ctypes.c_void_p(out.ctypes.data),
                                        ctypes.byref(inf), _stream_ptr(stream)))
        return out, _info_dict(inf)

    def close(self):
        if self._p:
            _lib.apc_blocks_free(self._p)
            self._p = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def select_pipeline(field, mode: str = "eb", stream=None) -> Scheme:
    assert field.is_cuda and field.is_contiguous()
    dims = (ctypes.c_int64 * field.dim())(*field.shape)
    s = _Scheme()
    _check(_lib.apc_select_pipeline(ctypes.c_void_p(field.data_ptr()), _dtype_code(field), dims, field.dim(),
                                    MODES[mode], ctypes.byref(s), _stream_ptr(stream)))
    return Scheme._from_c(s, field.dim())


def tune_tiles(field, degree: int = 3, stream=None) -> dict:
    """Time the per-level max and quantization sweeps with every tile width
    on this field and keep the fastest (or a wider one within 3% of it) for
    its level shapes (a process-wide table)."""
    assert field.is_cuda and field.is_contiguous()
    dims = (ctypes.c_int64 * field.dim())(*field.shape)
    t0 = ctypes.c_int32()
    us = (ctypes.c_double * 3)()
    _check(_lib.apc_tune_tiles(ctypes.c_void_p(field.data_ptr()), _dtype_code(field), dims, field.dim(), degree,
                               _stream_ptr(stream), ctypes.byref(t0), us))
    return {"tile": t0.value, "us": {32: us[0], 64: us[1], 128: us[2]}}


def tile_override(t2: int) -> None:
    """Force one sweep tile width (32, 64 or 128) for every pass; 0 = tuned/default."""
    _check(_lib.apc_tile_override(t2))


def tile_width(dtype, m1: int, m2: int) -> int:
    import torch
    t = ctypes.c_int32()
    _check(_lib.apc_tile_width(APC_F64 if dtype == torch.float64 else APC_F32, m1, m2, ctypes.byref(t)))
    return t.value


def axis_norms(n: int, L: int, degree: int) -> Tuple[List[float], List[float]]:
    """Host-only: exact 1D chain norms (max row / column abs sums) per level."""
    a = (ctypes.c_double * L)()
    b = (ctypes.c_double * L)()
    _check(_lib.apc_axis_norms(n, L, degree, a, b))
    return list(a), list(b)


def profile_enable(on: bool = True) -> None:
    _check(_lib.apc_profile_enable(1 if on else 0))


def profile_only(name=None) -> None:
    """Time only launches of this kernel name (None: every launch)."""
    _check(_lib.apc_profile_only(name.encode() if name else None))


def profile_report() -> dict:
    """Per-kernel launch counts, event-timed milliseconds and bytes moved."""
    ln = _i64()
    _check(_lib.apc_profile_report(None, 0, ctypes.byref(ln)))
    buf = ctypes.create_string_buffer(ln.value + 1)
    _check(_lib.apc_profile_report(buf, ln.value + 1, None))
    return json.loads(buf.value.decode())


def library():
    return _lib
