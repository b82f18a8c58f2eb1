"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

- The oracle is rebuilt with gcc's sanitizers and every pin runs against it
  in a process with the sanitizer runtime preloaded.
- The library is rebuilt with the sanitizers on its host code only (device
  code is unchanged; GPU sanitizers are not used), and a driver process
  runs its host-only paths: key expansion, key range checks and argument
  checks that fail before any device call. The key tables it expanded must
  equal the oracle's.
Any sanitizer report aborts the child process, which fails the test."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import oracle_pins

TESTS = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(TESTS)
GCC_ASAN = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
CLANG_ASAN = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

PINS_SCRIPT = """
import sys
sys.path[:0] = [{tests!r}, {root!r}]
import ctypes
import oracle, oracle_pins
assert hasattr(ctypes.CDLL(None), "__asan_init"), "sanitizer runtime not loaded"
o = oracle.load({lib!r})
for pin in oracle_pins.ALL_PINS:
    pin(o)
print("pins ok", len(oracle_pins.ALL_PINS), flush=True)
"""


def _child(cmd, preload, timeout):
    env = dict(os.environ, LD_PRELOAD=preload, **ENV_SAN)
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


@pytest.mark.skipif(not os.path.exists(GCC_ASAN), reason="gcc's AddressSanitizer runtime is not installed")
def test_oracle_pins_under_sanitizers(tmp_path):
    so = oracle.build(oracle.SRC, str(tmp_path / "liboracle_san.so"),
                      extra=("-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                             "-fno-sanitize-recover=undefined"))
    out = _child([sys.executable, "-c", PINS_SCRIPT.format(tests=TESTS, root=ROOT, lib=so)], GCC_ASAN, 600)
    assert "pins ok" in out


@pytest.mark.slow
@pytest.mark.skipif(not CLANG_ASAN, reason="clang's AddressSanitizer runtime is not installed")
def test_library_host_code_under_sanitizers(tmp_path, orc):
    from paper_1609_09840_amd import build

    flags = ("-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer")
    lib = build.build(lib=str(tmp_path / "libpmp_san.so"), build_dir=str(tmp_path / "_build"), extra=flags,
                      runtime_dir="/opt/rocm/lib")
    forced = [str(f[0]) for w in (False, True) for f in oracle_pins.reject_seeds(w)]
    npz = str(tmp_path / "keys.npz")
    out = _child([sys.executable, os.path.join(TESTS, "host_sanitizer_driver.py"), lib, npz, *forced],
                 CLANG_ASAN[-1], 600)
    assert "host driver ok" in out
    got = np.load(npz)
    assert len(got.files) >= 2 * (6 + len(forced))
    for name in got.files:
        bits, seed = name.split("_")
        want = orc.expand_keys32(int(seed)) if bits == "k32" else orc.expand_keys64(int(seed))
        assert np.array_equal(got[name], want), name
