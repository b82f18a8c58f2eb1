"""Test oracle for PM+32 / PM+64: a ctypes wrapper around ``pmp_oracle.c``.

THIS IS TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it. The GPU library never
imports, links or calls anything here, and nothing here imports the library.

The C file computes the paper's definitions with exact ``unsigned __int128``
arithmetic and plain ``%`` (Eq. (1), Algorithm 1, Sec. 4 byte padding, Sec. 5
output reduction, Sec. 7 mixers). See the header of ``pmp_oracle.c`` for the
readings of the paper it takes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pmp_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# output modes of the oracle (its own numbering; not shared with the library)
MIXED, RAW, FIELD = 0, 1, 2

P32 = (1 << 32) + 15
P64 = (1 << 64) + 13

_lib = None


def build(src: str = SRC, out: str = LIB, extra: tuple = ()) -> str:
    """Compile the oracle with gcc into a shared object and return its path."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-pthread", *extra, src, "-o", out]
    subprocess.run(cmd, check=True)
    return out


def _declare(lib):
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_splitmix64_stream.argtypes = [ctypes.c_uint64, u64p, ctypes.c_uint64]
    lib.oracle_splitmix64_stream.restype = None
    lib.oracle_expand_keys32.argtypes = [ctypes.c_uint64, ctypes.c_void_p]
    lib.oracle_expand_keys64.argtypes = [ctypes.c_uint64, ctypes.c_void_p]
    lib.oracle_mix32.argtypes = [ctypes.c_uint32]
    lib.oracle_mix32.restype = ctypes.c_uint32
    lib.oracle_mix64.argtypes = [ctypes.c_uint64]
    lib.oracle_mix64.restype = ctypes.c_uint64
    for name in ("oracle_pm32_words", "oracle_pm64_words"):
        getattr(lib, name).argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int, ctypes.c_int, u64p]
    for name in ("oracle_pm32", "oracle_pm64"):
        getattr(lib, name).argtypes = [ctypes.c_char_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int, u64p]
    lib.oracle_batch.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
    return lib


def load(path: str | None = None):
    """Load the oracle (building it first if the shared object is missing)."""
    global _lib
    if path is not None:
        return Oracle(_declare(ctypes.CDLL(path)))
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = Oracle(_declare(ctypes.CDLL(LIB)))
    return _lib


class OracleError(RuntimeError):
    pass


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """Python face of one loaded oracle shared object."""

    def __init__(self, lib):
        self.lib = lib

    # -- key material -------------------------------------------------------
    def splitmix64_stream(self, seed: int, n: int) -> np.ndarray:
        out = np.zeros(n, dtype=np.uint64)
        self.lib.oracle_splitmix64_stream(seed, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n)
        return out

    def expand_keys32(self, seed: int) -> np.ndarray:
        k = np.zeros(1032, dtype=np.uint32)
        self.lib.oracle_expand_keys32(seed, _ptr(k))
        return k

    def expand_keys64(self, seed: int) -> np.ndarray:
        k = np.zeros(1032, dtype=np.uint64)
        self.lib.oracle_expand_keys64(seed, _ptr(k))
        return k

    # -- mixers -------------------------------------------------------------
    def mix32(self, z: int) -> int:
        return int(self.lib.oracle_mix32(z))

    def mix64(self, z: int) -> int:
        return int(self.lib.oracle_mix64(z))

    # -- single strings -----------------------------------------------------
    def pm32(self, data: bytes, keys: np.ndarray, mode: int = MIXED) -> tuple[int, int]:
        """Return (value, levels). FIELD gives h in [0, p); RAW h mod 2^32."""
        keys = np.ascontiguousarray(keys, dtype=np.uint32)
        out = (ctypes.c_uint64 * 2)()
        r = self.lib.oracle_pm32(bytes(data), len(data), _ptr(keys), mode, out)
        if r < 0:
            raise OracleError(r)
        return int(out[0]), r

    def pm64(self, data: bytes, keys: np.ndarray, mode: int = MIXED) -> tuple[int, int]:
        """Return (value, levels). FIELD gives h in [0, p) as a Python int."""
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = (ctypes.c_uint64 * 2)()
        r = self.lib.oracle_pm64(bytes(data), len(data), _ptr(keys), mode, out)
        if r < 0:
            raise OracleError(r)
        v = int(out[0]) | (int(out[1]) << 64) if mode == FIELD else int(out[0])
        return v, r

    def words32(self, sigma, a, b, m: int, lmax: int) -> tuple[int, int]:
        sig = np.ascontiguousarray(sigma, dtype=np.uint64)
        a = np.ascontiguousarray(a, dtype=np.uint32)
        b = np.ascontiguousarray(b, dtype=np.uint32)
        out = (ctypes.c_uint64 * 2)()
        r = self.lib.oracle_pm32_words(_ptr(sig), len(sig), _ptr(a), _ptr(b), m, lmax, out)
        if r < 0:
            raise OracleError(r)
        return int(out[0]), r

    def words64(self, sigma, a, b, m: int, lmax: int) -> tuple[int, int]:
        sig = np.ascontiguousarray(sigma, dtype=np.uint64)
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        out = (ctypes.c_uint64 * 2)()
        r = self.lib.oracle_pm64_words(_ptr(sig), len(sig), _ptr(a), _ptr(b), m, lmax, out)
        if r < 0:
            raise OracleError(r)
        return int(out[0]) | (int(out[1]) << 64), r

    # -- batches ------------------------------------------------------------
    def batch(self, wide: bool, buf: np.ndarray, offsets: np.ndarray, keys: np.ndarray,
              mode: int = MIXED, nthreads: int = 1) -> np.ndarray:
        """Hash string i = buf[offsets[i]:offsets[i+1]] for all i.

        Returns uint32[count] (PM+32 mixed/raw), uint64[count] (PM+32 field,
        PM+64 mixed/raw) or uint64[count, 2] (PM+64 field: lo, hi)."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        keys = np.ascontiguousarray(keys, dtype=np.uint64 if wide else np.uint32)
        count = len(offsets) - 1
        stride = 2 if (wide and mode == FIELD) else 1
        out = np.zeros(count * stride, dtype=np.uint64)
        if buf.size == 0:
            buf = np.zeros(1, dtype=np.uint8)
        r = self.lib.oracle_batch(1 if wide else 0, _ptr(buf), _ptr(offsets), count, _ptr(keys), mode,
                                  _ptr(out), nthreads)
        if r < 0:
            raise OracleError(r)
        if wide and mode == FIELD:
            return out.reshape(count, 2)
        if not wide and mode != FIELD:
            return out.astype(np.uint32)
        return out
