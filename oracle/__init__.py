"""Python access to the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  The product library never imports it.  `build()` compiles
`hfx_oracle.c` with gcc/OpenMP into `_build/liboracle.so` next to this file.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# HFX_ORACLE_SO: load another build of the same source (the sanitizer build
# of the tests); it is never compiled here.
_SO = os.environ.get("HFX_ORACLE_SO") or os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "hfx_oracle.c")
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def build_sanitized(path: str) -> str:
    """Compile the oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    (every finding fatal) into `path`.  Loading it needs the ASan runtime
    preloaded into the process (LD_PRELOAD)."""
    os.makedirs(os.path.dirname(path), exist_ok=True)
    src = os.path.join(_HERE, "hfx_oracle.c")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           "-fno-sanitize-recover=undefined", "-o", path, src, "-lm"])
    return path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            if os.environ.get("HFX_ORACLE_SO"):
                raise FileNotFoundError(_SO)
            build(force=True)
        L = ctypes.CDLL(_SO)
        L.oracle_boys.restype = ctypes.c_double
        L.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double]
        basis = [_f64p, ctypes.c_int, _i32p, _i32p, _i32p, _i32p, _f64p, _f64p]
        L.oracle_normalise.restype = None
        L.oracle_normalise.argtypes = [ctypes.c_int, _i32p, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.oracle_shell_quartet.restype = ctypes.c_int
        L.oracle_shell_quartet.argtypes = basis + [ctypes.c_int] * 4 + [ctypes.c_double, _f64p]
        L.oracle_eri_tensor.restype = ctypes.c_int
        L.oracle_eri_tensor.argtypes = basis + [ctypes.c_double, _f64p]
        L.oracle_schwarz.restype = ctypes.c_int
        L.oracle_schwarz.argtypes = basis + [ctypes.c_double, _f64p]
        L.oracle_schwarz_list.restype = ctypes.c_int
        L.oracle_schwarz_list.argtypes = basis + [ctypes.c_double, ctypes.c_int64, _i64p, _f64p]
        L.oracle_build_K.restype = ctypes.c_int
        L.oracle_build_K.argtypes = basis + [_f64p, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                             _f64p, _f64p, _i64p]
        L.oracle_build_JK.restype = ctypes.c_int
        L.oracle_build_JK.argtypes = basis + [_f64p, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              _f64p, _f64p, _f64p, _i64p]
        L.oracle_build_JK_density.restype = ctypes.c_int
        L.oracle_build_JK_density.argtypes = basis + [_f64p, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                      ctypes.c_void_p, _f64p, _f64p, _i64p]
        L.oracle_build_K_periodic.restype = ctypes.c_int
        L.oracle_build_K_periodic.argtypes = basis + [ctypes.c_int, _f64p, ctypes.c_double, ctypes.c_double,
                                                      ctypes.c_int, _f64p, _i64p]
        L.oracle_digest_list.restype = ctypes.c_int
        L.oracle_digest_list.argtypes = basis + [_f64p, ctypes.c_double, ctypes.c_int64, _i64p,
                                                 ctypes.c_int, _f64p]
        L.oracle_class_index.restype = ctypes.c_int
        L.oracle_class_index.argtypes = [ctypes.c_int] * 4
        _lib = L
    return _lib


def _basis_args(sys):
    return (np.ascontiguousarray(sys.xyz, dtype=np.float64).ravel(), int(sys.nshell),
            np.ascontiguousarray(sys.shell_atom, dtype=np.int32),
            np.ascontiguousarray(sys.shell_l, dtype=np.int32),
            np.ascontiguousarray(sys.shell_nprim, dtype=np.int32),
            np.ascontiguousarray(sys.shell_off, dtype=np.int32),
            np.ascontiguousarray(sys.exps, dtype=np.float64),
            np.ascontiguousarray(sys.coefs, dtype=np.float64))


def boys(m: int, T: float) -> float:
    return lib().oracle_boys(int(m), float(T))


def normalised_coefs(sys) -> np.ndarray:
    out = np.zeros_like(np.asarray(sys.exps, dtype=np.float64))
    a = _basis_args(sys)
    lib().oracle_normalise(a[1], a[3], a[4], a[5], a[6], a[7], out)
    return out


def shell_quartet(sys, I, J, K, L, omega=0.0) -> np.ndarray:
    l = sys.shell_l
    shape = tuple(int(2 * l[s] + 1) for s in (I, J, K, L))
    out = np.zeros(int(np.prod(shape)), dtype=np.float64)
    rc = lib().oracle_shell_quartet(*_basis_args(sys), int(I), int(J), int(K), int(L), float(omega), out)
    if rc:
        raise ValueError("oracle_shell_quartet: invalid basis")
    return out.reshape(shape)


def eri_tensor(sys, omega=0.0) -> np.ndarray:
    n = sys.nbf
    out = np.zeros(n ** 4, dtype=np.float64)
    rc = lib().oracle_eri_tensor(*_basis_args(sys), float(omega), out)
    if rc:
        raise ValueError("oracle_eri_tensor: invalid basis")
    return out.reshape(n, n, n, n)


def schwarz(sys, omega=0.0) -> np.ndarray:
    npair = sys.nshell * (sys.nshell + 1) // 2
    Q = np.zeros(npair, dtype=np.float64)
    rc = lib().oracle_schwarz(*_basis_args(sys), float(omega), Q)
    if rc:
        raise ValueError("oracle_schwarz: invalid basis")
    return Q


def schwarz_list(sys, pids, omega=0.0) -> np.ndarray:
    """Schwarz factors of the listed pair indices p = I(I+1)/2 + J."""
    pids = np.ascontiguousarray(pids, dtype=np.int64)
    Q = np.zeros(len(pids), dtype=np.float64)
    rc = lib().oracle_schwarz_list(*_basis_args(sys), float(omega), len(pids), pids, Q)
    if rc:
        raise ValueError("oracle_schwarz_list: invalid basis")
    return Q


def build_K(sys, tau=1e-10, omega=0.0, nthreads=0, P=None):
    """Returns (K, Q, counts) with counts = dict(quartets, prim_quartets, per_class[21])."""
    n = sys.nbf
    P = np.ascontiguousarray(sys.P if P is None else P, dtype=np.float64)
    K = np.zeros((n, n), dtype=np.float64)
    npair = sys.nshell * (sys.nshell + 1) // 2
    Q = np.zeros(max(npair, 1), dtype=np.float64)
    cnt = np.zeros(23, dtype=np.int64)
    rc = lib().oracle_build_K(*_basis_args(sys), P.ravel(), float(tau), float(omega), int(nthreads),
                              K.ravel(), Q, cnt)
    if rc:
        raise ValueError("oracle_build_K: invalid basis")
    return K, Q[:npair], dict(quartets=int(cnt[0]), prim_quartets=int(cnt[1]),
                               per_class=cnt[2:].copy())


def build_JK(sys, tau=1e-10, omega=0.0, nthreads=0, P=None):
    """Coulomb J_ij = sum_kl (ij|kl) P_kl and exchange K from the same screened
    unique quartets.  Returns (J, K, Q, counts) as build_K."""
    n = sys.nbf
    P = np.ascontiguousarray(sys.P if P is None else P, dtype=np.float64)
    J = np.zeros((n, n), dtype=np.float64)
    K = np.zeros((n, n), dtype=np.float64)
    npair = sys.nshell * (sys.nshell + 1) // 2
    Q = np.zeros(max(npair, 1), dtype=np.float64)
    cnt = np.zeros(23, dtype=np.int64)
    rc = lib().oracle_build_JK(*_basis_args(sys), P.ravel(), float(tau), float(omega), int(nthreads),
                               J.ravel(), K.ravel(), Q, cnt)
    if rc:
        raise ValueError("oracle_build_JK: invalid basis")
    return J, K, Q[:npair], dict(quartets=int(cnt[0]), prim_quartets=int(cnt[1]),
                                  per_class=cnt[2:].copy())


def build_K_density(sys, tau=1e-10, omega=0.0, nthreads=0, P=None, coulomb=False):
    """Exchange build with the density-weighted test added to the Schwarz
    test (a quartet passing Q_IJ Q_KL >= tau is computed iff also
    Q_IJ Q_KL D >= tau, D = largest |P| over its digestion's shell blocks).
    coulomb=True: J as well (D then includes the blocks (I,J) and (K,L)).
    Returns (K, Q, counts), or (J, K, Q, counts) with coulomb=True."""
    n = sys.nbf
    P = np.ascontiguousarray(sys.P if P is None else P, dtype=np.float64)
    K = np.zeros((n, n), dtype=np.float64)
    J = np.zeros((n, n), dtype=np.float64) if coulomb else None
    npair = sys.nshell * (sys.nshell + 1) // 2
    Q = np.zeros(max(npair, 1), dtype=np.float64)
    cnt = np.zeros(23, dtype=np.int64)
    jp = J.ctypes.data_as(ctypes.c_void_p) if coulomb else None
    rc = lib().oracle_build_JK_density(*_basis_args(sys), P.ravel(), float(tau), float(omega), int(nthreads),
                                       jp, K.ravel(), Q, cnt)
    if rc:
        raise ValueError("oracle_build_JK_density: invalid basis")
    c = dict(quartets=int(cnt[0]), prim_quartets=int(cnt[1]), per_class=cnt[2:].copy())
    return (J, K, Q[:npair], c) if coulomb else (K, Q[:npair], c)


def build_K_periodic(cl, tau=1e-10, omega=0.0, nthreads=0):
    """Periodic exchange of a cluster laid out home cell first
    (cl.meta['nhome_shell'] shells): returns (Kout, counts) with Kout the rows
    of the home cell's functions, Kout[mu][b] = K^{cell(b)}_{mu f(b)}."""
    nhome = int(cl.meta["nhome_shell"])
    n = cl.nbf
    nh = int(np.sum(2 * cl.shell_l[:nhome] + 1))
    P = np.ascontiguousarray(cl.P, dtype=np.float64)
    K = np.zeros((nh, n), dtype=np.float64)
    cnt = np.zeros(23, dtype=np.int64)
    rc = lib().oracle_build_K_periodic(*_basis_args(cl), nhome, P.ravel(), float(tau), float(omega), int(nthreads),
                                       K.ravel(), cnt)
    if rc:
        raise ValueError("oracle_build_K_periodic: invalid basis")
    return K, dict(quartets=int(cnt[0]), prim_quartets=int(cnt[1]), per_class=cnt[2:].copy())


def digest_list(sys, pairs_pq: np.ndarray, omega=0.0, nthreads=0, P=None) -> np.ndarray:
    """K' (unsymmetrised) from an explicit list of unique quartets given as
    (p, q) pair indices with p >= q (pair index p = I(I+1)/2 + J, I >= J)."""
    n = sys.nbf
    P = np.ascontiguousarray(sys.P if P is None else P, dtype=np.float64)
    pq = np.ascontiguousarray(pairs_pq, dtype=np.int64).reshape(-1, 2)
    Kp = np.zeros((n, n), dtype=np.float64)
    rc = lib().oracle_digest_list(*_basis_args(sys), P.ravel(), float(omega), int(pq.shape[0]),
                                  pq.ravel(), int(nthreads), Kp.ravel())
    if rc:
        raise ValueError("oracle_digest_list: invalid basis")
    return Kp


def class_index(la, lb, lc, ld) -> int:
    return lib().oracle_class_index(la, lb, lc, ld)
