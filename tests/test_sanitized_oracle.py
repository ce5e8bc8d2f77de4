"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
every exported entry point runs on small systems in a child process with the
ASan runtime preloaded, any finding is fatal, and the results equal those of
the ordinary build."""

import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent(
    """
    import sys
    import numpy as np
    sys.path.insert(0, {root!r})
    import hfx_inputs as hi
    import oracle
    out = {{}}
    out["boys"] = np.array([oracle.boys(m, t) for m in range(9) for t in (0.0, 1e-3, 0.7, 12.0, 35.9, 36.0, 80.0)])
    s = hi.sp8_cluster()
    out["eri"] = oracle.eri_tensor(s, omega=0.11)
    out["Q"] = oracle.schwarz(s)
    J, K, _, c = oracle.build_JK(s, tau=1e-10, omega=0.11, nthreads=2)
    out["K"], out["J"] = K, J
    Kd, _, _ = oracle.build_K_density(s, tau=1e-8, omega=0.0, nthreads=2)
    out["Kd"] = Kd
    n = s.nshell
    pq = np.array([[p, q] for p in range(n * (n + 1) // 2) for q in range(p + 1)][:200], dtype=np.int64)
    out["dig"] = oracle.digest_list(s, pq, omega=0.11, nthreads=2)
    d = hi.lattice_system(2, seed=3, nprim_range=(1, 2))
    out["Kl"] = oracle.build_K(d, tau=1e-10, omega=0.11, nthreads=2)[0]
    cl = hi.periodic_cluster(natom_cell=1, reach=(1, 0, 0), lmax=1, nprim_range=(1, 2))
    out["Kp"] = oracle.build_K_periodic(cl, tau=1e-10, omega=0.11, nthreads=2)[0]
    np.savez(sys.argv[1], **out)
    print("done", flush=True)
    """
)


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no ASan runtime")
    so = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    script = tmp_path / "child.py"
    script.write_text(CHILD.format(root=ROOT))
    res = {}
    # the runtime goes first; whatever the environment already preloads stays
    pre = asan + (":" + os.environ["LD_PRELOAD"] if os.environ.get("LD_PRELOAD") else "")
    for tag, extra in (("san", {"HFX_ORACLE_SO": so, "LD_PRELOAD": pre,
                                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0",
                                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}),
                       ("plain", {})):
        env = dict(os.environ, **extra)
        if tag == "plain":
            env.pop("HFX_ORACLE_SO", None)
        out = tmp_path / f"{tag}.npz"
        r = subprocess.run([sys.executable, str(script), str(out)], env=env, capture_output=True, text=True,
                           timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
        res[tag] = np.load(out)
    for k in res["plain"].files:
        a, b = res["san"][k], res["plain"][k]
        assert a.shape == b.shape, k
        assert np.allclose(a, b, rtol=1e-13, atol=1e-15), k


def test_sanitizer_harness_reports_a_planted_overflow(tmp_path):
    """Control for the test above: the same flags and preload catch a heap
    overflow planted in a throwaway C function (CPU only)."""
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no ASan runtime")
    src = tmp_path / "bad.c"
    src.write_text("#include <stdlib.h>\n"
                   "double bad(int n) { double *a = malloc(n * sizeof(double)); double s = 0;\n"
                   "  for (int i = 0; i <= n; ++i) a[i] = i;  /* one past the end */\n"
                   "  for (int i = 0; i < n; ++i) s += a[i]; free(a); return s; }\n")
    so = tmp_path / "libbad.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-fPIC", "-shared", "-fsanitize=address,undefined",
                           "-fno-omit-frame-pointer", "-o", str(so), str(src)])
    code = ("import ctypes; L = ctypes.CDLL(%r); L.bad.restype = ctypes.c_double; L.bad(7)" % str(so))
    pre = asan + (":" + os.environ["LD_PRELOAD"] if os.environ.get("LD_PRELOAD") else "")
    env = dict(os.environ, LD_PRELOAD=pre, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr
