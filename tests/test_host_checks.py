"""Argument checks of the newer entry points, which run on the host before
any device call (CPU only: the fake device pointers below are never
dereferenced)."""
from __future__ import annotations

import ctypes
import os

import pytest

from paper_1609_09840_amd import build

if not os.path.exists(build.LIB):
    pytest.skip("libpmp.so is not built", allow_module_level=True)

from paper_1609_09840_amd import pmp  # noqa: E402

L = pmp._lib
FAKE = ctypes.c_void_p(0x10000)  # never read: every call below fails its checks first


def batch(count=4, wide=0, flags=0, keys=0x20000):
    return pmp.pmp_batch(buf=0x30000, buf_bytes=100, offsets=0x40000, count=count, keys=keys, out=0x50000,
                         flags=flags, wide=wide)


def test_hash128_checks():
    assert L.pmp_hash128(FAKE, 100, FAKE, -1, FAKE, FAKE, 0, FAKE, 1 << 20, None) == pmp.PMP_E_INVALID_ARG
    assert L.pmp_hash128(FAKE, 100, None, 4, FAKE, FAKE, 0, FAKE, 1 << 20, None) == pmp.PMP_E_INVALID_ARG
    assert L.pmp_hash128(FAKE, 100, FAKE, 4, FAKE, FAKE, 8, FAKE, 1 << 20, None) == pmp.PMP_E_INVALID_ARG
    need = L.pmp_hash128_scratch_bytes(4, 100)
    assert L.pmp_hash128(FAKE, 100, FAKE, 4, FAKE, FAKE, 0, FAKE, need - 1, None) == pmp.PMP_E_INVALID_ARG
    assert "scratch" in pmp.pmp_last_error()
    assert L.pmp_hash128(FAKE, 100, FAKE, 0, FAKE, FAKE, 0, FAKE, 0, None) == pmp.PMP_OK  # nothing to do


def test_hash128_scratch_grows_with_input():
    a = L.pmp_hash128_scratch_bytes(1000, 1 << 20)
    assert L.pmp_hash128_scratch_bytes(2000, 1 << 20) > a
    assert L.pmp_hash128_scratch_bytes(1000, 1 << 30) > a
    assert L.pmp_hash128_scratch_bytes(-1, 0) == 0


def test_table_checks():
    b = batch()
    m = 1024
    w = L.pmp_table_work_bytes(m)
    assert w >= 4 * m
    assert L.pmp_table_build(None, None, m, FAKE, FAKE, FAKE, w, None) == pmp.PMP_E_INVALID_ARG
    assert L.pmp_table_build(None, ctypes.byref(b), 0, FAKE, FAKE, FAKE, w, None) == pmp.PMP_E_INVALID_ARG
    assert L.pmp_table_build(None, ctypes.byref(b), m, FAKE, FAKE, FAKE, w - 1, None) == pmp.PMP_E_INVALID_ARG
    bf = batch(flags=pmp.PMP_OUT_FIELD)
    assert L.pmp_table_build(None, ctypes.byref(bf), m, FAKE, FAKE, FAKE, w, None) == pmp.PMP_E_INVALID_ARG
    q64 = batch(wide=1)
    assert L.pmp_table_probe(None, ctypes.byref(q64), ctypes.byref(b), m, FAKE, FAKE, FAKE, None) == \
        pmp.PMP_E_INVALID_ARG  # variants differ
    qk = batch(keys=0x60000)
    assert L.pmp_table_probe(None, ctypes.byref(qk), ctypes.byref(b), m, FAKE, FAKE, FAKE, None) == \
        pmp.PMP_E_INVALID_ARG  # key tables differ
    assert "share" in pmp.pmp_last_error()


def test_incr_checks():
    assert L.pmp_incr_append(None, FAKE, 10) == pmp.PMP_E_INVALID_ARG
    assert L.pmp_incr_digest(None, FAKE, 0) == pmp.PMP_E_INVALID_ARG
    assert L.pmp_incr_reset(None) == pmp.PMP_E_INVALID_ARG
    assert L.pmp_incr_destroy(None) == pmp.PMP_OK
    out = ctypes.c_void_p()
    assert L.pmp_incr_create(2, FAKE, None, ctypes.byref(out)) == pmp.PMP_E_INVALID_ARG
    assert L.pmp_incr_create(0, None, None, ctypes.byref(out)) == pmp.PMP_E_INVALID_ARG
