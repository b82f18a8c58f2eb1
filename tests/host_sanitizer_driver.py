"""Runs the library's host-only code paths (key expansion, key range checks,
argument checks that fail before any device call) from a library built with
AddressSanitizer and UndefinedBehaviorSanitizer on its host code. Started by
test_sanitizers.py in a process of its own with the sanitizer runtime
preloaded; it loads the library with ctypes only (no PyTorch, no GPU) and
writes the key tables it expanded to an .npz file for the parent to compare
with the oracle.

usage: python host_sanitizer_driver.py <library.so> <out.npz>
"""
import ctypes
import sys

import numpy as np

assert hasattr(ctypes.CDLL(None), "__asan_init"), "sanitizer runtime not loaded"
lib = ctypes.CDLL(sys.argv[1])
vp = ctypes.c_void_p
FAKE = vp(0x10000)  # never dereferenced: every call below fails its checks first
E_INVALID_ARG = -1
E_KEY_RANGE = -2

lib.pmp_last_error.restype = ctypes.c_char_p
lib.pmp_version.restype = ctypes.c_char_p
lib.pmp_hash128_scratch_bytes.restype = ctypes.c_uint64
lib.pmp_hash128_scratch_bytes.argtypes = [ctypes.c_int64, ctypes.c_uint64]
lib.pmp_table_work_bytes.restype = ctypes.c_uint64
lib.pmp_table_work_bytes.argtypes = [ctypes.c_uint64]
lib.pmp_hash128.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_int64, vp, vp, ctypes.c_uint32, vp, ctypes.c_uint64, vp]
lib.pmp_incr_append.argtypes = [vp, vp, ctypes.c_uint64]
for name in ("pmp_expand_keys32", "pmp_expand_keys64", "pmp_expand_keys128"):
    getattr(lib, name).argtypes = [ctypes.c_uint64, vp]

tables = {}
for seed in (0, 1, 2, 7, 12345, 2**64 - 1) + tuple(int(s) for s in sys.argv[3:]):
    k32 = np.zeros(1032, np.uint32)
    k64 = np.zeros(1032, np.uint64)
    k128 = np.zeros(2064, np.uint64)
    assert lib.pmp_expand_keys32(seed, k32.ctypes.data) == 0
    assert lib.pmp_expand_keys64(seed, k64.ctypes.data) == 0
    assert lib.pmp_expand_keys128(seed, k128.ctypes.data) == 0
    assert lib.pmp_check_keys32(vp(k32.ctypes.data)) == 0
    assert lib.pmp_check_keys64(vp(k64.ctypes.data)) == 0
    assert lib.pmp_check_keys128(vp(k128.ctypes.data)) == 0
    k32[5] = 2**32 - 13
    k64[1023] = 2**64 - 11
    assert lib.pmp_check_keys32(vp(k32.ctypes.data)) == E_KEY_RANGE
    assert lib.pmp_check_keys64(vp(k64.ctypes.data)) == E_KEY_RANGE
    assert lib.pmp_last_error()
    k32[:] = 0
    k64[:] = 0
    lib.pmp_expand_keys32(seed, k32.ctypes.data)
    lib.pmp_expand_keys64(seed, k64.ctypes.data)
    tables[f"k32_{seed}"], tables[f"k64_{seed}"] = k32, k64

# argument checks that return before any device call
assert lib.pmp_hash128(FAKE, 100, FAKE, -1, FAKE, FAKE, 0, FAKE, 1 << 20, None) == E_INVALID_ARG
assert lib.pmp_hash128(FAKE, 100, None, 4, FAKE, FAKE, 0, FAKE, 1 << 20, None) == E_INVALID_ARG
assert lib.pmp_hash128_scratch_bytes(-1, 0) == 0
assert lib.pmp_hash128_scratch_bytes(1000, 1 << 20) > 0
assert lib.pmp_table_work_bytes(1024) >= 4096
assert lib.pmp_incr_append(None, FAKE, 10) == E_INVALID_ARG
assert lib.pmp_incr_reset(None) == E_INVALID_ARG
assert lib.pmp_incr_destroy(None) == 0
out = vp()
assert lib.pmp_incr_create(2, FAKE, None, ctypes.byref(out)) == E_INVALID_ARG
assert lib.pmp_version()
np.savez(sys.argv[2], **tables)
print("host driver ok", len(tables), "tables", flush=True)
