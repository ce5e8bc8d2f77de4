"""Mixed precision: quartets whose FP32 error scale E_IJ E_KL is below the
cut are evaluated in FP32 (FP32 records, Boys table and recurrences; large-T
Boys, centres, horizontal recurrence and accumulation in FP64), the rest in
FP64.

Stated bar: max |K_mixed - K_oracle| <= 1e-6 hartree at the default cut 1e-5
(measured 1.1e-10 on the 128-atom subset of the 1024-atom lattice).  This
part has no pin beyond the FP64 oracle: its accuracy is measured.
"""

import sys

import numpy as np
import pytest

import hfx_inputs as hi
import oracle
import paper_2009_03559_amd as hfx

pytestmark = pytest.mark.gpu
CUT = hfx.MIXED_CUT  # default FP32 cut
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(s, o):
    p = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    K = torch.empty_like(P)
    st = hfx.build_K(p, P, K, o, stats=True)
    torch.cuda.synchronize()
    return K.cpu().numpy(), st


def _count_split(Q, tau, cut):
    qq = np.outer(Q, Q)
    tri = np.tril(np.ones_like(qq, dtype=bool))
    n64 = int(((qq >= max(tau, cut)) & tri).sum())
    n32 = int(((qq >= tau) & (qq < cut) & tri).sum())
    return n64, n32


@pytest.mark.parametrize("omega", [0.0, hi.OMEGA_HSE])
def test_mixed_vs_oracle_dzp(omega):
    s = hi.lattice_system(8, seed=23, nprim_range=(1, 3))
    Ko, Q, cnt = oracle.build_K(s, tau=1e-10, omega=omega)
    Km, st = _run(s, hfx.opts(tau=1e-10, omega=omega, prec=hfx.PREC_MIXED, mixed_cut=CUT))
    err = np.abs(Km - Ko).max()
    trerr = abs(np.trace(s.P @ Km) - np.trace(s.P @ Ko))
    _say("mixed dzp8", omega, "max|dK|", err, "tr(PK) err", trerr, "fp32", st["quartets_fp32"], "/", st["quartets"])
    assert err <= 1e-6
    assert st["quartets"] == cnt["quartets"]
    # FP32 where the quartet's FP32 error scale E_IJ E_KL (>= Q_IJ Q_KL) is
    # below the cut: a subset of the quartets whose bound is below it
    n64, n32 = _count_split(Q, 1e-10, CUT)
    assert 0 < st["quartets_fp32"] <= n32
    assert st["quartets"] - st["quartets_fp32"] >= n64


def test_mixed_cut_zero_is_fp64():
    s = hi.sp8_cluster()
    K64, _ = _run(s, hfx.opts(tau=1e-10, omega=0.11))
    Km, st = _run(s, hfx.opts(tau=1e-10, omega=0.11, prec=hfx.PREC_MIXED, mixed_cut=0.0))
    assert st["quartets_fp32"] == 0
    assert np.abs(Km - K64).max() <= 1e-13


def test_all_fp32_error_is_bounded_and_measured():
    """Cut above every bound: every quartet in FP32 -- still FP64 accumulation."""
    s = hi.sp8_cluster()
    Ko, _, cnt = oracle.build_K(s, tau=1e-10, omega=0.11)
    Km, st = _run(s, hfx.opts(tau=1e-10, omega=0.11, prec=hfx.PREC_MIXED, mixed_cut=1e30))
    err = np.abs(Km - Ko).max()
    _say("all-FP32 sp8_cluster max|dK|", err, "max|K|", np.abs(Ko).max())
    assert st["quartets_fp32"] == cnt["quartets"]
    assert err <= 1e-5 * np.abs(Ko).max()


def test_mixed_vs_fp64_gpu_larger():
    """24-atom DZP lattice (the 256-atom lattice recipe at reduced size): mixed vs the
    FP64 GPU path (itself held to the oracle above)."""
    s = hi.lattice_system(24, seed=2)
    K64, st64 = _run(s, hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE))
    Km, stm = _run(s, hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE, prec=hfx.PREC_MIXED, mixed_cut=CUT))
    err = np.abs(Km - K64).max()
    _say("mixed vs fp64 lattice24: max|dK|", err, "fp32 frac", stm["quartets_fp32"] / stm["quartets"],
         "t64", st64["device_s"], "tmix", stm["device_s"])
    assert stm["quartets"] == st64["quartets"]
    assert err <= 1e-6


def test_mixed_translated_32_atoms_full_contraction():
    """32 atoms of the benchmark lattice recipe with its 3-6 primitives per
    shell, moved 24-40 bohr away from the coordinate origin (FP32 rounding of
    absolute centres would show here): mixed vs the FP64 GPU path within the
    stated 1e-6 hartree (margin printed), and the FP64 path itself
    translation invariant."""
    s = hi.lattice_system(32, seed=5)
    t = hi.lattice_system(32, seed=5)
    t.xyz = t.xyz + np.array([24.0, 20.0, 16.0])
    o64 = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    om = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE, prec=hfx.PREC_MIXED, mixed_cut=CUT)
    K0, st0 = _run(s, o64)
    K64, st64 = _run(t, o64)
    Km, stm = _run(t, om)
    e_tr = np.abs(K64 - K0).max()
    err = np.abs(Km - K64).max()
    trerr = abs(np.sum(t.P * Km) - np.sum(t.P * K64))
    _say("translated lattice32: FP64 translation diff", e_tr, "mixed vs FP64 max|dK|", err,
         "margin x%.1f" % (1e-6 / max(err, 1e-300)), "tr(PK) err", trerr,
         "fp32 frac", stm["quartets_fp32"] / stm["quartets"])
    assert st64["quartets"] == st0["quartets"] == stm["quartets"]
    assert e_tr <= 1e-10
    assert err <= 1e-6
