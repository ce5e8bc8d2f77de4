"""Coulomb J from the same quartets as K (hfx_build_JK): J and K against the
oracle's joint build on the same seeded systems, FP64 bar 1e-10 hartree;
mixed precision within the mixed bar; K from the joint build equals the
K-only build up to the order of the atomics."""

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
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def _gpu_JK(s, o):
    p = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    J, K = torch.empty_like(P), torch.empty_like(P)
    st = hfx.build_JK(p, P, J, K, o, stats=True)
    K1 = torch.empty_like(P)
    hfx.build_K(p, P, K1, o)
    torch.cuda.synchronize()
    return J.cpu().numpy(), K.cpu().numpy(), K1.cpu().numpy(), st


@pytest.mark.parametrize("omega", [0.0, hi.OMEGA_HSE])
def test_JK_sp8_cluster(omega):
    s = hi.sp8_cluster()
    _say("JK sp8_cluster omega", omega)
    J, K, K1, st = _gpu_JK(s, hfx.opts(tau=1e-10, omega=omega))
    Jo, Ko, _, cnt = oracle.build_JK(s, tau=1e-10, omega=omega)
    assert np.abs(J - Jo).max() <= 1e-10
    assert np.abs(K - Ko).max() <= 1e-10
    assert np.abs(K - K1).max() <= 1e-12
    assert np.abs(J - J.T).max() == 0.0
    assert st["quartets"] == cnt["quartets"]


@pytest.mark.parametrize("prim_tau", [0.0, None])
@pytest.mark.parametrize("omega", [0.0, hi.OMEGA_HSE])
@pytest.mark.parametrize("tau", [0.0, 1e-10])
def test_JK_dzp_small(tau, omega, prim_tau):
    """8-atom DZP lattice: every class pair, split and unsplit classes."""
    s = hi.lattice_system(8, seed=23, nprim_range=(1, 3))
    _say("JK dzp8 tau", tau, "omega", omega, "prim_tau", prim_tau)
    J, K, K1, st = _gpu_JK(s, hfx.opts(tau=tau, omega=omega, prim_tau=prim_tau))
    Jo, Ko, _, cnt = oracle.build_JK(s, tau=tau, omega=omega)
    assert np.abs(J - Jo).max() <= 1e-10, np.abs(J - Jo).max()
    assert np.abs(K - Ko).max() <= 1e-10
    assert np.abs(K - K1).max() <= 1e-12
    assert st["quartets"] == cnt["quartets"]


def test_JK_mixed():
    s = hi.lattice_system(8, seed=23, nprim_range=(1, 3))
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE, prec=hfx.PREC_MIXED)
    J, K, _, st = _gpu_JK(s, o)
    Jo, Ko, _, _ = oracle.build_JK(s, tau=1e-10, omega=hi.OMEGA_HSE)
    _say("JK mixed max|dJ|", np.abs(J - Jo).max(), "max|dK|", np.abs(K - Ko).max(), "fp32", st["quartets_fp32"])
    assert st["quartets_fp32"] > 0
    assert np.abs(J - Jo).max() <= 1e-6
    assert np.abs(K - Ko).max() <= 1e-6


def test_JK_segmented_and_shard_free(monkeypatch):
    """J through the segmented launch path equals the single-launch J."""
    s = hi.lattice_system(12, seed=31, nprim_range=(1, 3))
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    J1, _, _, _ = _gpu_JK(s, o)
    monkeypatch.setenv("HFX_MAX_BLOCKS", "1")
    J2, _, _, _ = _gpu_JK(s, o)
    monkeypatch.delenv("HFX_MAX_BLOCKS")
    assert np.abs(J1 - J2).max() <= 1e-12 * max(1.0, np.abs(J1).max())


def test_JK_rejects_aliasing():
    s = hi.sp8_cluster()
    o = hfx.opts(omega=0.11)
    p = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    K = torch.empty_like(P)
    for J in (K, P):
        with pytest.raises(hfx.HfxError) as e:
            hfx.build_JK(p, P, J, K, o)
        assert e.value.status == hfx.HFX_EINVAL


@pytest.mark.parametrize("nshards", [3, 7])
def test_shards_sum_to_full_build(nshards):
    """hfx_build_K_shard / hfx_build_JK_shard: the bra slots of every class are
    dealt round-robin; the symmetrised partial matrices of all shards add up
    to the single-device J and K, and the quartet counts add up too."""
    s = hi.lattice_system(8, seed=23, nprim_range=(1, 3))
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    p = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    J, K = torch.empty_like(P), torch.empty_like(P)
    st = hfx.build_JK(p, P, J, K, o, stats=True)
    Js, Ks = torch.zeros_like(P), torch.zeros_like(P)
    Kk = torch.zeros_like(P)
    nq = 0
    for sh in range(nshards):
        Jp, Kp = torch.empty_like(P), torch.empty_like(P)
        nq += hfx.build_JK_shard(p, P, Jp, Kp, o, sh, nshards, stats=True)["quartets"]
        Js += Jp
        Ks += Kp
        K1 = torch.empty_like(P)
        hfx.build_K_shard(p, P, K1, o, sh, nshards)
        Kk += K1
    torch.cuda.synchronize()
    assert nq == st["quartets"]
    assert torch.abs(Js - J).max().item() <= 1e-12 * max(1.0, torch.abs(J).max().item())
    assert torch.abs(Ks - K).max().item() <= 1e-12 * max(1.0, torch.abs(K).max().item())
    assert torch.abs(Kk - K).max().item() <= 1e-12 * max(1.0, torch.abs(K).max().item())
    with pytest.raises(hfx.HfxError) as e:
        hfx.build_K_shard(p, P, Kk, o, nshards, nshards)
    assert e.value.status == hfx.HFX_EINVAL


def test_JK_leading_dimension():
    s = hi.sp8_cluster()
    n = s.nbf
    big = torch.zeros((n, n + 5), dtype=torch.float64, device="cuda")
    big[:, :n] = torch.from_numpy(s.P).cuda()
    Jb = torch.full((n, n + 5), 3.0, dtype=torch.float64, device="cuda")
    Kb = torch.full((n, n + 5), 7.0, dtype=torch.float64, device="cuda")
    o = hfx.opts(omega=0.11)
    p = hfx.pairs_from_system(s, o)
    hfx.build_JK(p, big[:, :n], Jb[:, :n], Kb[:, :n], o)
    torch.cuda.synchronize()
    Jo, Ko, _, _ = oracle.build_JK(s, tau=1e-10, omega=0.11)
    Jg, Kg = Jb.cpu().numpy(), Kb.cpu().numpy()
    assert np.abs(Jg[:, :n] - Jo).max() <= 1e-10
    assert np.abs(Kg[:, :n] - Ko).max() <= 1e-10
    assert (Jg[:, n:] == 3.0).all() and (Kg[:, n:] == 7.0).all()
