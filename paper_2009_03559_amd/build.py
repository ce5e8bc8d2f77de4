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


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-4000:]}")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    """Generate, compile and link; returns the library path."""
    os.makedirs(GEN, exist_ok=True)
    os.makedirs(OBJ, exist_ok=True)
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_eri.py"), "--outdir", GEN,
                           "--model", os.path.join(GEN, "model.json")])
    srcs = sorted(os.path.join(GEN, f) for f in os.listdir(GEN) if f.endswith(".hip"))
    srcs += [os.path.join(CSRC, f) for f in ("hfx_host.hip", "hfx_serve.hip")]
    # largest classes first so the pool finishes together (a class's
    # Coulomb-digesting variant shares its header)
    def header(src):
        return src.replace("tu_", "eri_").replace("_jk.hip", ".hip").replace(".hip", ".h")

    srcs.sort(key=lambda s: -os.path.getsize(header(s)) if os.path.exists(header(s)) else 0)
    jobs = jobs or min(16, os.cpu_count() or 4)
    objs = []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for o in ex.map(_compile, srcs):
            objs.append(o)
            if verbose:
                print("compiled", os.path.basename(o), flush=True)
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
