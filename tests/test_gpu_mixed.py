"""Mixed precision: quartets whose Schwarz bound Q_IJ Q_KL is below the cut
are evaluated in FP32 (FP32 records, Boys table and recurrences; large-T
Boys in FP64), the rest in FP64; all accumulation into K is FP64.

Stated bar: max |K_mixed - K_oracle| <= 1e-6 hartree at the tuned cut 1e-7.
At cut 1e-5 the measured error is ~2e-5 and at 1e-6 ~1.7e-6 on the 256-atom
shard (above the bar), so the cut is tuned to 1e-7.  This part has no pin beyond
the FP64 oracle: its accuracy is measured.
"""

import sys

import numpy as np
import pytest

import hfx_inputs as hi
import oracle
import paper_2009_03559_amd as hfx

pytestmark = pytest.mark.gpu
CUT = hfx.MIXED_CUT  # tuned FP32 cut
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
    n64, n32 = _count_split(Q, 1e-10, CUT)
    assert st["quartets_fp32"] == n32 and st["quartets"] - st["quartets_fp32"] == n64
    assert st["quartets_fp32"] > 0


def test_mixed_cut_zero_is_fp64():
    s = hi.config0()
    K64, _ = _run(s, hfx.opts(tau=1e-10, omega=0.11))
    Km, st = _run(s, hfx.opts(tau=1e-10, omega=0.11, prec=hfx.PREC_MIXED, mixed_cut=0.0))
    assert st["quartets_fp32"] == 0
    assert np.abs(Km - K64).max() <= 1e-13


def test_all_fp32_error_is_bounded_and_measured():
    """Cut above every bound: every quartet in FP32 -- still FP64 accumulation."""
    s = hi.config0()
    Ko, _, cnt = oracle.build_K(s, tau=1e-10, omega=0.11)
    Km, st = _run(s, hfx.opts(tau=1e-10, omega=0.11, prec=hfx.PREC_MIXED, mixed_cut=1e30))
    err = np.abs(Km - Ko).max()
    _say("all-FP32 config0 max|dK|", err, "max|K|", np.abs(Ko).max())
    assert st["quartets_fp32"] == cnt["quartets"]
    assert err <= 1e-5 * np.abs(Ko).max()


def test_mixed_vs_fp64_gpu_larger():
    """24-atom DZP lattice (the config-1 recipe at reduced size): mixed vs the
    FP64 GPU path (itself held to the oracle above)."""
    s = hi.lattice_system(24, seed=2)
    K64, st64 = _run(s, hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE))
    Km, stm = _run(s, hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE, prec=hfx.PREC_MIXED, mixed_cut=CUT))
    err = np.abs(Km - K64).max()
    _say("mixed vs fp64 lattice24: max|dK|", err, "fp32 frac", stm["quartets_fp32"] / stm["quartets"],
         "t64", st64["device_s"], "tmix", stm["device_s"])
    assert stm["quartets"] == st64["quartets"]
    assert err <= 1e-6
