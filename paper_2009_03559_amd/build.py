"""Build libhfx.so for gfx950 in-tree (paper_2009_03559_amd/_build/).

Steps: generate the per-class device code with csrc/gen_eri.py, compile every
translation unit with hipcc in parallel, link one shared library.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.environ.get("HFX_BUILD_DIR") or os.path.join(HERE, "_build")
GEN = os.path.join(BUILD, "gen")
OBJ = os.path.join(BUILD, "obj")
LIB = os.path.join(BUILD, "libhfx.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-I" + GEN]


# HFX_HOST_SANITIZE=1: AddressSanitizer and UndefinedBehaviorSanitizer on the
# host code of the runtime (device code unchanged).  The library does not
# link the sanitizer runtime: the program that loads it provides it (an
# executable built with the same sanitizers, or a preloaded shared runtime).
HOST_SANITIZE = os.environ.get("HFX_HOST_SANITIZE") == "1"
HOST_SOURCES = ("hfx_host.hip", "hfx_serve.hip", "hfx_noalloc.hip")
SAN_FLAGS = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


COMMON_HEADERS = [os.path.join(CSRC, "hfx_device.hpp"), os.path.join(CSRC, "hfx_internal.hpp"),
                  os.path.join(ROOT, "include", "hfx.h")]


def _header_of(src: str) -> str:
    return src.replace("tu_", "eri_").replace("_jk.hip", ".hip").replace("_per.hip", ".hip").replace(".hip", ".h")


def _stale(src: str) -> bool:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return True
    deps = [src] + COMMON_HEADERS
    h = _header_of(src)
    if os.path.exists(h):
        deps.append(h)
    return max(os.path.getmtime(d) for d in deps) > os.path.getmtime(obj)


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    extra = SAN_FLAGS if HOST_SANITIZE and os.path.basename(src) in HOST_SOURCES else []
    cmd = [HIPCC] + FLAGS + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-4000:]}")
    return obj


def build(jobs: int | None = None, verbose: bool = True, only_changed: bool = False) -> str:
    """Generate, compile and link; returns the library path.  only_changed:
    recompile only translation units older than their sources (development
    builds); the default compiles everything."""
    os.makedirs(GEN, exist_ok=True)
    os.makedirs(OBJ, exist_ok=True)
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_eri.py"), "--outdir", GEN,
                           "--model", os.path.join(GEN, "model.json")])
    srcs = sorted(os.path.join(GEN, f) for f in os.listdir(GEN) if f.endswith(".hip"))
    srcs += [os.path.join(CSRC, f) for f in HOST_SOURCES]
    # largest classes first so the pool finishes together (a class's
    # Coulomb-digesting variant shares its header)
    srcs.sort(key=lambda s: -os.path.getsize(_header_of(s)) if os.path.exists(_header_of(s)) else 0)
    todo = [s for s in srcs if _stale(s) or (HOST_SANITIZE and os.path.basename(s) in HOST_SOURCES)] \
        if only_changed else srcs
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        for o in ex.map(_compile, todo):
            if verbose:
                print("compiled", os.path.basename(o), flush=True)
    objs = [os.path.join(OBJ, os.path.basename(s) + ".o") for s in srcs]
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(only_changed="--changed" in sys.argv)
