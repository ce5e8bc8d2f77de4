"""Density-weighted exchange screening on the GPU against the oracle's
density-screened build: a quartet that passes Q_IJ Q_KL >= tau is computed
only if Q_IJ Q_KL D >= tau as well, D the largest |P| over the shell blocks
its digestion multiplies.  Bars: the screened quartet counts per class equal
the oracle's exactly; K (and J) within 1e-10 hartree; mixed precision within
1e-6; batched K equal to the solo K."""

import os
import sys

import numpy as np
import pytest

import hfx_inputs as hi
import oracle
import paper_2009_03559_amd as hfx

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device(tmp_path_factory):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    os.environ["HFX_TUNE_CACHE"] = str(tmp_path_factory.mktemp("tune") / "autotune.txt")


def _gpu(s, o, coulomb=False, prim_tau=None):
    p = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    K = torch.empty_like(P)
    if coulomb:
        J = torch.empty_like(P)
        st = hfx.build_JK(p, P, J, K, o, stats=True)
        torch.cuda.synchronize()
        return J.cpu().numpy(), K.cpu().numpy(), st
    st = hfx.build_K(p, P, K, o, stats=True)
    torch.cuda.synchronize()
    return K.cpu().numpy(), st


@pytest.mark.parametrize("omega", [0.0, hi.OMEGA_HSE])
@pytest.mark.parametrize("case", ["sp8_cluster", "dzp8", "dzp6_full"])
def test_density_K_equals_oracle(case, omega):
    if case == "sp8_cluster":
        s, tau = hi.sp8_cluster(), 1e-10
    elif case == "dzp8":
        s, tau = hi.lattice_system(8, seed=23, nprim_range=(1, 3)), 1e-8
    else:  # the workload's 3-6 primitives per shell
        s, tau = hi.lattice_system(6, seed=31), 1e-10
    _say("density K", case, omega)
    Ko, _, cnt = oracle.build_K_density(s, tau=tau, omega=omega)
    _, _, c0 = oracle.build_K(s, tau=tau, omega=omega)
    Kg, st = _gpu(s, hfx.opts(tau=tau, omega=omega, density=True))
    err = np.abs(Kg - Ko).max()
    _say("  quartets", st["quartets"], "of", c0["quartets"], "(Schwarz only); max |dK|", err)
    assert err <= 1e-10
    assert st["quartets"] == cnt["quartets"]
    assert list(st["class_quartets"]) == list(cnt["per_class"])
    assert np.abs(Kg - Kg.T).max() == 0.0


def test_density_JK_equals_oracle():
    s = hi.lattice_system(8, seed=23, nprim_range=(1, 3))
    tau = 1e-8
    Jo, Ko, _, cnt = oracle.build_K_density(s, tau=tau, omega=hi.OMEGA_HSE, coulomb=True)
    Jg, Kg, st = _gpu(s, hfx.opts(tau=tau, omega=hi.OMEGA_HSE, density=True), coulomb=True)
    _say("density JK: quartets", st["quartets"], "max |dJ|", np.abs(Jg - Jo).max(), "max |dK|", np.abs(Kg - Ko).max())
    assert st["quartets"] == cnt["quartets"]
    assert np.abs(Jg - Jo).max() <= 1e-10
    assert np.abs(Kg - Ko).max() <= 1e-10


def test_density_mixed_within_bar():
    s = hi.lattice_system(8, seed=23, nprim_range=(1, 3))
    tau = 1e-10
    Ko, _, cnt = oracle.build_K_density(s, tau=tau, omega=hi.OMEGA_HSE)
    Km, st = _gpu(s, hfx.opts(tau=tau, omega=hi.OMEGA_HSE, density=True, prec=hfx.PREC_MIXED))
    err = np.abs(Km - Ko).max()
    _say("density mixed: max |dK|", err, "fp32", st["quartets_fp32"], "of", st["quartets"])
    assert st["quartets"] == cnt["quartets"]
    assert err <= 1e-6


def test_density_tiles_span_many_candidates():
    """A 16-atom lattice at a loose tau: long ket ranges, most candidates
    dropped by the density test, survivors queued across many 64-wide
    candidate chunks; K equals the Schwarz-only K within the dropped
    quartets' bound, counts equal a second build, and the batch path gives
    the same K."""
    s = hi.lattice_system(16, seed=41, nprim_range=(1, 2))
    tau = 1e-6
    od = hfx.opts(tau=tau, omega=hi.OMEGA_HSE, density=True)
    K1, st1 = _gpu(s, od)
    K0, st0 = _gpu(s, hfx.opts(tau=tau, omega=hi.OMEGA_HSE))
    _say("density 16 atoms: quartets", st1["quartets"], "of", st0["quartets"])
    assert st1["quartets"] < st0["quartets"]
    Kd, _, cnt = oracle.build_K_density(s, tau=tau, omega=hi.OMEGA_HSE)
    assert st1["quartets"] == cnt["quartets"]
    assert np.abs(K1 - Kd).max() <= 1e-10
    p = hfx.pairs_from_system(s, od)
    P = torch.from_numpy(s.P).cuda()
    Kb = torch.empty_like(P)
    stb = hfx.build_K_batch([p], [P], [Kb], od, stats=True)
    torch.cuda.synchronize()
    assert stb["quartets"] == st1["quartets"]
    assert np.abs(Kb.cpu().numpy() - K1).max() <= 1e-12


def test_unknown_flag_rejected():
    s = hi.sp8_cluster()
    o = hfx.opts()
    o.flags = 6
    with pytest.raises(hfx.HfxError) as e:
        hfx.pairs_from_system(s, o)
    assert e.value.status == hfx.HFX_EINVAL
