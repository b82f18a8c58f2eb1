"""Build libpmp.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpmp.so")
SOURCES = ["pmp_kernels.hip", "pmp_static.hip", "pmp_incr.hip", "pmp_table.hip", "pmp_pm128.hip", "pmp_probe.hip", "pmp_api.cpp", "pmp_server.cpp"]
HEADERS = ["pmp_device.hpp", "pmp_internal.h", "pmp_batch.h", "pmp_incr.h", "pmp_stage.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
BUILD_DIR = os.path.join(PKG, "_build")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed fp32 instructions stay off (none are needed for integer work)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # private arrays stay in registers; LDS is reserved for the staging buffers
    "-mllvm", "-disable-promote-alloca-to-lds",
    "-I" + INCLUDE,
    "-I" + CSRC,
]


def hip_runtime_dir() -> str:
    """Directory of the HIP runtime the process will use. PyTorch wheels carry
    their own libamdhip64.so; linking libpmp.so to that same file keeps one HIP
    runtime per process (two runtimes cannot share devices, pointers or
    streams). Without PyTorch the ROCm installation is used."""
    try:
        import importlib.util

        spec = importlib.util.find_spec("torch")
        if spec and spec.origin:
            d = os.path.join(os.path.dirname(spec.origin), "lib")
            if os.path.exists(os.path.join(d, "libamdhip64.so")):
                return d
    except Exception:
        pass
    return "/opt/rocm/lib"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln)
    if res.returncode != 0:
        raise RuntimeError(f"{cmd[0]} failed ({res.returncode}):\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)


def build(verbose: bool = False, lib: str = LIB, build_dir: str = BUILD_DIR, extra: tuple = (),
          runtime_dir: str | None = None, jobs: int = 0) -> str:
    """Compile every source and link the library (always recompiles). ``extra``
    adds compiler flags (a host-sanitizer build passes its flags here, each
    behind -Xarch_host, into a build directory and library path of its own);
    sources compile in parallel on ``jobs`` threads (default: one per
    source, at most the host's CPU count)."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(build_dir, exist_ok=True)
    objs = [os.path.join(build_dir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1))
    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    rt = runtime_dir or hip_runtime_dir()
    tmp = lib + ".tmp"
    link = ["g++", "-shared", "-o", tmp, *objs, "-L" + rt, "-l:libamdhip64.so", "-Wl,-rpath," + rt, "-pthread",
            "-Wl,-z,now"]
    if not extra:
        link.append("-Wl,--no-undefined")  # a sanitizer build takes its runtime from LD_PRELOAD
    _run(link, verbose)
    os.replace(tmp, lib)
    return lib


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [os.path.join(INCLUDE, "pmp.h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    print(build(verbose=True))
