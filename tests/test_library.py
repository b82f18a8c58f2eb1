"""The C-ABI library (CPU only, no compute calls): it loads, exports every
function include/pmp.h declares, and the binding refuses to work without it."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmp.h")


def declared_functions() -> list[str]:
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|uint64_t|const char\s*\*)\s+(pmp_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("pmp_hash32", "pmp_hash64", "pmp_expand_keys32", "pmp_expand_keys64", "pmp_check_keys32",
                 "pmp_check_keys64", "pmp_hash_mixed", "pmp_hash_many", "pmp_plan_create", "pmp_server_create",
                 "pmp_last_error", "pmp_incr_create", "pmp_incr_append", "pmp_incr_digest", "pmp_table_build",
                 "pmp_table_probe", "pmp_table_work_bytes", "pmp_hash128", "pmp_hash128_scratch_bytes",
                 "pmp_expand_keys128"):
        assert must in names, must


def test_library_exports_every_declared_symbol():
    from paper_1609_09840_amd import build

    if not os.path.exists(build.LIB):
        pytest.skip("libpmp.so is not built")
    import torch  # noqa: F401  (same HIP runtime as the binding uses)

    lib = ctypes.CDLL(build.LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_calls_work_without_a_gpu():
    """Key expansion and checks are host code: they run here."""
    from paper_1609_09840_amd import build

    if not os.path.exists(build.LIB):
        pytest.skip("libpmp.so is not built")
    from paper_1609_09840_amd import pmp

    k32 = pmp.pmp_expand_keys32(1)
    k64 = pmp.pmp_expand_keys64(2)
    assert pmp.pmp_check_keys32(k32) == pmp.PMP_OK and pmp.pmp_check_keys64(k64) == pmp.PMP_OK
    k32[5] = 0xFFFFFFFF
    assert pmp.pmp_check_keys32(k32) == pmp.PMP_E_KEY_RANGE
    assert pmp.pmp_version().startswith("pmp")


def test_binding_fails_loudly_without_the_library():
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1609_09840_amd.build as b\n"
            "b.LIB = '/nonexistent/libpmp.so'\n"
            "try:\n"
            "    import paper_1609_09840_amd.pmp\n"
            "except ImportError as e:\n"
            "    print('refused:', e); sys.exit(0)\n"
            "sys.exit(3)\n") % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "refused" in r.stdout, (r.returncode, r.stdout, r.stderr)
