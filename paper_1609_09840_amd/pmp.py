"""Python binding of libpmp (ctypes): the C ABI of include/pmp.h with the same
names. It only marshals arguments; every hash step runs in the library's HIP
kernels. PyTorch supplies device memory and streams.

The library must be built (``python -m paper_1609_09840_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

PMP_OK = 0
PMP_E_INVALID_ARG = -1
PMP_E_KEY_RANGE = -2
PMP_E_TOO_LONG = -3
PMP_E_OFFSETS = -4
PMP_E_HIP = -5
PMP_E_NOMEM = -6
PMP_NOALLOC_SCRATCH_BYTES = 16 << 20  # include/pmp.h
PMP_E_INTERNAL = -7
PMP_ALPHA_BY_COUNT = 0xFFFFFFFF  # pmp_plan_tune: split batches by string count

PMP_NO_MIX = 1
PMP_OUT_FIELD = 2
PMP_KEYS = 1032


class PmpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pmp error {code}: {msg}")
        self.code = code


class pmp_batch(ctypes.Structure):
    _fields_ = [
        ("buf", ctypes.c_void_p),
        ("buf_bytes", ctypes.c_uint64),
        ("offsets", ctypes.c_void_p),
        ("count", ctypes.c_int64),
        ("keys", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
        ("wide", ctypes.c_uint32),
    ]


class pmp_server_config(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int),
        ("lanes", ctypes.c_int),
        ("lane_bytes", ctypes.c_uint64),
        ("d_keys32", ctypes.c_void_p),
        ("d_keys64", ctypes.c_void_p),
        ("max_requests_per_batch", ctypes.c_int),
        ("max_batch_strings", ctypes.c_int64),
        ("reserve_bytes", ctypes.c_uint64),
        ("max_inflight_bytes", ctypes.c_uint64),
        ("idle_spin_us", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class pmp_request(ctypes.Structure):
    _fields_ = [
        ("buf", ctypes.c_void_p),
        ("buf_bytes", ctypes.c_uint64),
        ("offsets", ctypes.c_void_p),
        ("count", ctypes.c_int64),
        ("out", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
        ("wide", ctypes.c_uint32),
        ("device_resident", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class pmp_tuning(ctypes.Structure):
    _fields_ = [
        ("g32", ctypes.c_int32),
        ("g64", ctypes.c_int32),
        ("alpha", ctypes.c_uint32),
        ("waves_per_cu", ctypes.c_int32),
        ("shares_per_wave", ctypes.c_int32),
        ("ms", ctypes.c_float),
    ]


class pmp_server_report(ctypes.Structure):
    _fields_ = [
        ("completed", ctypes.c_uint64),
        ("rejected", ctypes.c_uint64),
        ("batches", ctypes.c_uint64),
        ("bytes", ctypes.c_uint64),
        ("failed", ctypes.c_uint64),
        ("p50_us", ctypes.c_double),
        ("p99_us", ctypes.c_double),
        ("max_us", ctypes.c_double),
        ("mean_us", ctypes.c_double),
        ("span_us", ctypes.c_double),
    ]


def _load():
    if not os.path.exists(_build.LIB):
        raise ImportError(f"libpmp.so is not built ({_build.LIB}); run __graft_entry__.build()")
    # Load PyTorch's HIP runtime first so that libpmp.so binds to the same
    # runtime instance (one per process) instead of a second copy.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(_build.LIB)
    vp, u64, i64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int
    sig = {
        "pmp_expand_keys32": [u64, vp],
        "pmp_expand_keys64": [u64, vp],
        "pmp_check_keys32": [vp],
        "pmp_check_keys64": [vp],
        "pmp_plan_create": [i32, ctypes.POINTER(vp)],
        "pmp_plan_destroy": [vp],
        "pmp_plan_reserve": [vp, u64, i64],
        "pmp_plan_status": [vp, vp],
        "pmp_plan_set_tile": [vp, i32, i32],
        "pmp_plan_tune": [vp, i32, u32, u64, i32],
        "pmp_probe_mad_rate": [ctypes.POINTER(ctypes.c_double)],
        "pmp_probe_read_bw": [vp, u64, ctypes.POINTER(ctypes.c_double)],
        "pmp_hash32": [vp, vp, u64, vp, i64, vp, vp, u32, vp],
        "pmp_hash64": [vp, vp, u64, vp, i64, vp, vp, u32, vp],
        "pmp_hash_mixed": [vp, ctypes.POINTER(pmp_batch), ctypes.POINTER(pmp_batch), vp],
        "pmp_hash_mixed_noalloc": [ctypes.POINTER(pmp_batch), ctypes.POINTER(pmp_batch), vp, vp],
        "pmp_hash_many": [vp, ctypes.POINTER(pmp_batch), i32, vp],
        "pmp_graph_create": [vp, ctypes.POINTER(pmp_batch), i32, ctypes.POINTER(vp)],
        "pmp_graph_launch": [vp, vp],
        "pmp_graph_destroy": [vp],
        "pmp_plan_autotune": [vp, ctypes.POINTER(pmp_batch), i32, vp, ctypes.POINTER(pmp_tuning)],
        "pmp_server_create": [ctypes.POINTER(pmp_server_config), ctypes.POINTER(vp)],
        "pmp_server_destroy": [vp],
        "pmp_server_submit": [vp, ctypes.POINTER(pmp_request), ctypes.POINTER(u64)],
        "pmp_server_wait": [vp, u64, i64],
        "pmp_server_stats": [vp, ctypes.POINTER(pmp_server_report)],
        "pmp_server_reset_stats": [vp],
        "pmp_server_replay": [vp, ctypes.POINTER(pmp_request), i64, vp, vp],
        "pmp_server_status": [vp],
        "pmp_hash_plain": [i32, vp, u64, vp, i64, vp, vp, u32, vp, u64, vp],
        "pmp_debug_fold": [i32, vp, vp, vp, vp, i64, vp],
        "pmp_expand_keys128": [u64, vp],
        "pmp_check_keys128": [vp],
        "pmp_hash128": [vp, u64, vp, i64, vp, vp, u32, vp, u64, vp],
        "pmp_table_build": [vp, ctypes.POINTER(pmp_batch), u64, vp, vp, vp, u64, vp],
        "pmp_table_probe": [vp, ctypes.POINTER(pmp_batch), ctypes.POINTER(pmp_batch), u64, vp, vp, vp, vp],
        "pmp_incr_create": [i32, vp, vp, ctypes.POINTER(vp)],
        "pmp_incr_reserve": [vp, u64],
        "pmp_incr_append": [vp, vp, u64],
        "pmp_incr_digest": [vp, vp, u32],
        "pmp_incr_reset": [vp],
        "pmp_incr_length": [vp, ctypes.POINTER(u64)],
        "pmp_incr_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.pmp_hash128_scratch_bytes.argtypes = [i64, u64]
    lib.pmp_hash128_scratch_bytes.restype = u64
    lib.pmp_table_work_bytes.argtypes = [u64]
    lib.pmp_table_work_bytes.restype = u64
    lib.pmp_last_error.restype = ctypes.c_char_p
    lib.pmp_version.restype = ctypes.c_char_p
    return lib


_lib = _load()
LIB_PATH = _build.LIB


def _check(rc: int) -> int:
    if rc != PMP_OK:
        raise PmpError(rc, _lib.pmp_last_error().decode())
    return rc


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev_ptr(t, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def pmp_version() -> str:
    return _lib.pmp_version().decode()


def pmp_last_error() -> str:
    return _lib.pmp_last_error().decode()


# -- keys ------------------------------------------------------------------
def pmp_expand_keys32(seed: int) -> np.ndarray:
    k = np.zeros(PMP_KEYS, dtype=np.uint32)
    _check(_lib.pmp_expand_keys32(seed, k.ctypes.data_as(ctypes.c_void_p)))
    return k


def pmp_expand_keys64(seed: int) -> np.ndarray:
    k = np.zeros(PMP_KEYS, dtype=np.uint64)
    _check(_lib.pmp_expand_keys64(seed, k.ctypes.data_as(ctypes.c_void_p)))
    return k


def pmp_expand_keys128(seed: int) -> np.ndarray:
    """PM+128 key table: 2064 uint64, entries (lo, hi), a[8][128] then b[8]."""
    k = np.zeros(2 * PMP_KEYS, dtype=np.uint64)
    _check(_lib.pmp_expand_keys128(seed, k.ctypes.data_as(ctypes.c_void_p)))
    return k


def pmp_check_keys128(keys: np.ndarray) -> int:
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    return _lib.pmp_check_keys128(k.ctypes.data_as(ctypes.c_void_p))


def pmp_check_keys32(keys: np.ndarray) -> int:
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    return _lib.pmp_check_keys32(k.ctypes.data_as(ctypes.c_void_p))


def pmp_check_keys64(keys: np.ndarray) -> int:
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    return _lib.pmp_check_keys64(k.ctypes.data_as(ctypes.c_void_p))


# -- plans -----------------------------------------------------------------
class Plan:
    """Owned plan (workspace + status word) on one device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(_lib.pmp_plan_create(device, ctypes.byref(h)))
        self.handle = h

    def reserve(self, max_buf_bytes: int, max_count: int):
        _check(_lib.pmp_plan_reserve(self.handle, max_buf_bytes, max_count))

    def set_tile(self, wide: bool, lanes_per_block: int):
        _check(_lib.pmp_plan_set_tile(self.handle, int(wide), lanes_per_block))

    def tune(self, waves_per_cu: int = 0, alpha: int = 0, wave_bytes: int = 0, shares_per_wave: int = 0):
        _check(_lib.pmp_plan_tune(self.handle, waves_per_cu, alpha, wave_bytes, shares_per_wave))

    def status(self, stream=None) -> int:
        return _lib.pmp_plan_status(self.handle, _stream(stream))

    def close(self):
        if self.handle:
            _check(_lib.pmp_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pmp_plan_create(device: int = 0) -> Plan:
    return Plan(device)


def pmp_plan_status(plan: Plan | None = None, stream=None) -> int:
    return _lib.pmp_plan_status(plan.handle if plan else None, _stream(stream))


def _plan_ptr(plan):
    return plan.handle if plan is not None else None


# -- hashing ---------------------------------------------------------------
def _out_for(wide: bool, count: int, flags: int, device):
    import torch

    if flags & PMP_OUT_FIELD:
        return torch.empty(count * (2 if wide else 1), dtype=torch.uint64, device=device)
    return torch.empty(count, dtype=torch.uint64 if wide else torch.uint32, device=device)


def _hash(wide, buf, offsets, keys, out, flags, stream, plan, buf_bytes):
    import torch

    count = offsets.numel() - 1
    if out is None:
        out = _out_for(wide, count, flags, offsets.device)
    if buf_bytes is None:
        buf_bytes = buf.numel()
    if keys.dtype != (torch.uint64 if wide else torch.uint32) or keys.numel() != PMP_KEYS:
        raise ValueError("keys must be a device tensor of 1032 uint32 (PM+32) or uint64 (PM+64)")
    if offsets.dtype != torch.int64:
        raise ValueError("offsets must be int64")
    f = _lib.pmp_hash64 if wide else _lib.pmp_hash32
    bp = _dev_ptr(buf, "buf") if buf.numel() else ctypes.c_void_p(0)
    _check(f(_plan_ptr(plan), bp, buf_bytes, _dev_ptr(offsets, "offsets"), count, _dev_ptr(keys, "keys"),
             _dev_ptr(out, "out"), flags, _stream(stream)))
    return out


def pmp_hash32(buf, offsets, keys, out=None, flags: int = 0, stream=None, plan: Plan | None = None,
               buf_bytes: int | None = None):
    """PM+32 of string i = buf[offsets[i]:offsets[i+1]] for every i (device
    tensors: uint8 buf, int64 offsets, uint32[1032] keys). Returns out."""
    return _hash(False, buf, offsets, keys, out, flags, stream, plan, buf_bytes)


def pmp_hash64(buf, offsets, keys, out=None, flags: int = 0, stream=None, plan: Plan | None = None,
               buf_bytes: int | None = None):
    """PM+64 counterpart of pmp_hash32 (uint64[1032] keys)."""
    return _hash(True, buf, offsets, keys, out, flags, stream, plan, buf_bytes)


def pmp_hash128(buf, offsets, keys, out=None, flags: int = 0, scratch=None, stream=None,
                buf_bytes: int | None = None):
    """PM+128 of string i = buf[offsets[i]:offsets[i+1]] (device tensors:
    uint8 buf, int64 offsets, uint64[2064] keys). out: count x 2 uint64
    (h mod 2^128, low half first) or, with PMP_OUT_FIELD, count x 3."""
    import torch

    count = offsets.numel() - 1
    if buf_bytes is None:
        buf_bytes = buf.numel()
    if keys.dtype != torch.uint64 or keys.numel() != 2 * PMP_KEYS:
        raise ValueError("keys must be a device tensor of 2064 uint64")
    if out is None:
        out = torch.empty(count * (3 if flags & PMP_OUT_FIELD else 2), dtype=torch.uint64, device=offsets.device)
    need = int(_lib.pmp_hash128_scratch_bytes(count, buf_bytes))
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(max(need, 8), dtype=torch.uint8, device=offsets.device)
    bp = _dev_ptr(buf, "buf") if buf.numel() else ctypes.c_void_p(0)
    _check(_lib.pmp_hash128(bp, buf_bytes, _dev_ptr(offsets, "offsets"), count, _dev_ptr(keys, "keys"),
                            _dev_ptr(out, "out"), flags, _dev_ptr(scratch, "scratch"), scratch.numel(),
                            _stream(stream)))
    return out


def make_batch(wide: bool, buf, offsets, keys, out, flags: int = 0, buf_bytes: int | None = None) -> pmp_batch:
    return pmp_batch(
        buf=(buf.data_ptr() if buf.numel() else 0),
        buf_bytes=buf.numel() if buf_bytes is None else buf_bytes,
        offsets=offsets.data_ptr(),
        count=offsets.numel() - 1,
        keys=keys.data_ptr(),
        out=out.data_ptr(),
        flags=flags,
        wide=1 if wide else 0,
    )


def pmp_hash_mixed(b0: pmp_batch | None, b1: pmp_batch | None, stream=None, plan: Plan | None = None):
    """Both batches in one kernel launch (see make_batch)."""
    p0 = ctypes.byref(b0) if b0 is not None else None
    p1 = ctypes.byref(b1) if b1 is not None else None
    _check(_lib.pmp_hash_mixed(_plan_ptr(plan), p0, p1, _stream(stream)))


def pmp_hash_mixed_noalloc(b0, b1, status, stream=None):
    """pmp_hash_mixed on the library's static scratch (no allocation by the
    library); `status` is a device int32 tensor of one element that receives
    the status bits."""
    _check(_lib.pmp_hash_mixed_noalloc(ctypes.byref(b0) if b0 is not None else None,
                                       ctypes.byref(b1) if b1 is not None else None,
                                       _dev_ptr(status, "status"), _stream(stream)))


def pmp_hash_many(batches, stream=None, plan: Plan | None = None):
    """Any number of batches (list of pmp_batch) in one kernel launch."""
    arr = (pmp_batch * max(1, len(batches)))(*batches)
    _check(_lib.pmp_hash_many(_plan_ptr(plan), arr, len(batches), _stream(stream)))


class Graph:
    """A captured pmp_hash_many launch (pmp_graph_*), replayed by launch()."""

    def __init__(self, plan: Plan, batches):
        self._keep = (plan, list(batches))
        arr = (pmp_batch * max(1, len(batches)))(*batches)
        h = ctypes.c_void_p()
        _check(_lib.pmp_graph_create(plan.handle, arr, len(batches), ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(_lib.pmp_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if self.handle:
            _check(_lib.pmp_graph_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pmp_plan_autotune(plan: Plan, batches, stream=None) -> dict:
    """Time the compiled tile pairs and launch shapes on these batches and
    keep the fastest in the plan; returns the chosen setting."""
    arr = (pmp_batch * max(1, len(batches)))(*batches)
    t = pmp_tuning()
    _check(_lib.pmp_plan_autotune(plan.handle, arr, len(batches), _stream(stream), ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in pmp_tuning._fields_}


# -- serving ---------------------------------------------------------------
def _host_ptr(a: np.ndarray, name: str):
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError(f"{name} must be C-contiguous")
    return a.ctypes.data if a.size else 0


class Incr:
    """Incremental hash of one string appended in pieces (pmp_incr_*): the
    digest of the pieces so far equals pmp_hash32/64 of their concatenation.
    keys: device key table (uint32 or uint64 [1032]); every call is queued on
    `stream` (default: the current stream when the object is made)."""

    def __init__(self, wide: bool, keys, stream=None):
        import torch

        if keys.dtype != (torch.uint64 if wide else torch.uint32) or keys.numel() != PMP_KEYS:
            raise ValueError("keys must be a device tensor of 1032 uint32 (PM+32) or uint64 (PM+64)")
        self.wide = bool(wide)
        self.keys = keys  # kept alive: the library holds its pointer
        self.device = keys.device
        h = ctypes.c_void_p()
        _check(_lib.pmp_incr_create(int(wide), _dev_ptr(keys, "keys"), _stream(stream), ctypes.byref(h)))
        self.handle = h

    def reserve(self, max_piece_bytes: int):
        _check(_lib.pmp_incr_reserve(self.handle, max_piece_bytes))

    def append(self, piece, nbytes: int | None = None):
        """Append a device uint8 tensor (or `nbytes` bytes at its start). The
        tensor must stay unchanged until the stream has passed the call."""
        n = piece.numel() if nbytes is None else int(nbytes)
        if n > piece.numel():
            raise ValueError("nbytes exceeds the tensor")
        p = _dev_ptr(piece, "piece") if n else ctypes.c_void_p(0)
        _check(_lib.pmp_incr_append(self.handle, p, n))

    def digest(self, out=None, flags: int = 0):
        """Hash of everything appended so far (one output, layout as for
        pmp_hash32/64 with these flags); the state is kept."""
        if out is None:
            out = _out_for(self.wide, 1, flags, self.device)
        _check(_lib.pmp_incr_digest(self.handle, _dev_ptr(out, "out"), flags))
        return out

    def reset(self):
        _check(_lib.pmp_incr_reset(self.handle))

    def __len__(self):
        v = ctypes.c_uint64()
        _check(_lib.pmp_incr_length(self.handle, ctypes.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "handle", None):
            _check(_lib.pmp_incr_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Table:
    """Hash table over the strings of one batch (pmp_table_*): bucket =
    hash mod nbuckets, CSR arrays on the device. The key batch (and its
    tensors) is kept: probes read its bytes and hashes."""

    def __init__(self, wide: bool, buf, offsets, keys, nbuckets: int, flags: int = 0, stream=None,
                 plan: Plan | None = None):
        import torch

        if flags & PMP_OUT_FIELD:
            raise ValueError("a table keys on n-bit outputs (no PMP_OUT_FIELD)")
        count = offsets.numel() - 1
        dev = offsets.device
        self.wide, self.flags, self.nbuckets, self.plan = bool(wide), flags, int(nbuckets), plan
        self.tensors = (buf, offsets, keys)
        self.hashes = _out_for(wide, count, flags, dev)
        self.batch = make_batch(wide, buf, offsets, keys, self.hashes, flags)
        self.bucket_start = torch.empty(self.nbuckets + 1, dtype=torch.int64, device=dev)
        # one record per key: index, hash, offset, length (int64 each)
        self.entries = torch.empty((max(count, 1), 4), dtype=torch.int64, device=dev)
        nw = int(_lib.pmp_table_work_bytes(self.nbuckets))
        self.work = torch.empty(max(nw, 8), dtype=torch.uint8, device=dev)
        _check(_lib.pmp_table_build(_plan_ptr(plan), ctypes.byref(self.batch), self.nbuckets,
                                    _dev_ptr(self.bucket_start, "bucket_start"), _dev_ptr(self.entries, "entries"),
                                    _dev_ptr(self.work, "work"), nw, _stream(stream)))

    def probe(self, qbuf, qoffsets, out=None, qhashes=None, stream=None):
        """Smallest key index equal to each query's bytes, or -1 (int64)."""
        import torch

        n = qoffsets.numel() - 1
        dev = qoffsets.device
        if qhashes is None:
            qhashes = _out_for(self.wide, n, self.flags, dev)
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
        qb = make_batch(self.wide, qbuf, qoffsets, self.tensors[2], qhashes, self.flags)
        _check(_lib.pmp_table_probe(_plan_ptr(self.plan), ctypes.byref(qb), ctypes.byref(self.batch), self.nbuckets,
                                    _dev_ptr(self.bucket_start, "bucket_start"), _dev_ptr(self.entries, "entries"),
                                    _dev_ptr(out, "out"), _stream(stream)))
        return out[:n]


def pmp_table_build(wide: bool, buf, offsets, keys, nbuckets: int, flags: int = 0, stream=None,
                    plan: Plan | None = None) -> Table:
    return Table(wide, buf, offsets, keys, nbuckets, flags, stream, plan)


def pmp_incr_create(wide: bool, keys, stream=None) -> Incr:
    return Incr(wide, keys, stream)


class Server:
    """Continuous-batching server (pmp_server_*). Requests are hashed with the
    key tables given here (device tensors, uint32[1032] and uint64[1032])."""

    def __init__(self, keys32, keys64, device: int = 0, lanes: int = 2, lane_bytes: int = 64 << 20,
                 max_requests_per_batch: int = 256, max_batch_strings: int = 0, reserve_bytes: int = 0,
                 max_inflight_bytes: int = 0, idle_spin_us: int = 200):
        self._keys = (keys32, keys64)  # keep the tables alive
        cfg = pmp_server_config(device=device, lanes=lanes, lane_bytes=lane_bytes,
                                d_keys32=_dev_ptr(keys32, "keys32"), d_keys64=_dev_ptr(keys64, "keys64"),
                                max_requests_per_batch=max_requests_per_batch,
                                max_batch_strings=max_batch_strings, reserve_bytes=reserve_bytes,
                                max_inflight_bytes=max_inflight_bytes, idle_spin_us=idle_spin_us)
        h = ctypes.c_void_p()
        _check(_lib.pmp_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._live = {}

    @staticmethod
    def request(wide: bool, buf, offsets, out, flags: int = 0) -> pmp_request:
        """A request over numpy arrays (host: staged through a lane arena) or
        device tensors (hashed in place). The arrays must outlive the request."""
        import torch

        if isinstance(buf, torch.Tensor):
            return pmp_request(buf=buf.data_ptr() if buf.numel() else 0, buf_bytes=buf.numel(),
                               offsets=offsets.data_ptr(), count=offsets.numel() - 1, out=out.data_ptr(),
                               flags=flags, wide=int(wide), device_resident=1)
        return pmp_request(buf=_host_ptr(buf, "buf"), buf_bytes=buf.size, offsets=_host_ptr(offsets, "offsets"),
                           count=len(offsets) - 1, out=_host_ptr(out, "out"), flags=flags, wide=int(wide),
                           device_resident=0)

    def submit(self, req: pmp_request, keep=None) -> int:
        t = ctypes.c_uint64()
        _check(_lib.pmp_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        self._live[t.value] = keep
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1) -> int:
        rc = _lib.pmp_server_wait(self.handle, ticket, timeout_us)
        if rc == 1:
            return rc
        self._live.pop(ticket, None)
        return _check(rc)

    def replay(self, reqs, arrival_us: np.ndarray) -> np.ndarray:
        """Submit reqs[k] at arrival_us[k] (microseconds from the start), wait
        for all; returns each request's latency in microseconds."""
        n = len(reqs)
        arr = (pmp_request * max(1, n))(*reqs)
        at = np.ascontiguousarray(arrival_us, dtype=np.float64)
        lat = np.zeros(n, dtype=np.float64)
        _check(_lib.pmp_server_replay(self.handle, arr, n, at.ctypes.data_as(ctypes.c_void_p),
                                      lat.ctypes.data_as(ctypes.c_void_p)))
        return lat

    def stats(self) -> dict:
        r = pmp_server_report()
        _check(_lib.pmp_server_stats(self.handle, ctypes.byref(r)))
        return {f: getattr(r, f) for f, _ in pmp_server_report._fields_}

    def reset_stats(self):
        _check(_lib.pmp_server_reset_stats(self.handle))

    def status(self) -> int:
        return _lib.pmp_server_status(self.handle)

    def close(self):
        if self.handle:
            _check(_lib.pmp_server_destroy(self.handle))
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pmp_hash_plain(wide: bool, buf, h_offsets: np.ndarray, keys, out, flags: int, scratch, stream=None):
    """Baseline: one string per launch sequence (host offsets)."""
    h = np.ascontiguousarray(h_offsets, dtype=np.int64)
    _check(_lib.pmp_hash_plain(int(wide), _dev_ptr(buf, "buf"), buf.numel(), h.ctypes.data_as(ctypes.c_void_p),
                               len(h) - 1, _dev_ptr(keys, "keys"), _dev_ptr(out, "out"), flags,
                               _dev_ptr(scratch, "scratch"), scratch.numel() * scratch.element_size(),
                               _stream(stream)))
    return out


def pmp_probe_read_bw(buf) -> float:
    """Bytes per second a plain streaming read kernel reaches over the device
    tensor `buf` (at least 1 MiB)."""
    r = ctypes.c_double()
    _check(_lib.pmp_probe_read_bw(_dev_ptr(buf, "buf"), buf.numel() * buf.element_size(), ctypes.byref(r)))
    return r.value


def pmp_probe_mad_rate() -> float:
    """v_mad_u64_u32 lane operations per second on the current device (the
    multiply roofline)."""
    r = ctypes.c_double(0.0)
    _check(_lib.pmp_probe_mad_rate(ctypes.byref(r)))
    return r.value


def pmp_debug_fold(wide: bool, w0, w1, w2, z, stream=None):
    n = w2.numel()
    _check(_lib.pmp_debug_fold(int(wide), _dev_ptr(w0, "w0"), _dev_ptr(w1, "w1"), _dev_ptr(w2, "w2"),
                               _dev_ptr(z, "z"), n, _stream(stream)))
    return z
