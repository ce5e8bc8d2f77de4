"""Periodic exchange on the GPU against the oracle's periodic build: a crystal
written as a cluster of image cells (home cell first), K^G for the home
cell's rows, the lattice sums over the cluster's cells.  Bars: K within
1e-10 hartree element by element; the screened (home pair, pair) counts per
class equal the oracle's."""

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


def _gpu(cl, tau, omega, prim_tau=None):
    o = hfx.opts(tau=tau, omega=omega, prim_tau=prim_tau)
    p = hfx.pairs_from_system(cl, o)
    nhs = int(cl.meta["nhome_shell"])
    nh = int(np.sum(2 * cl.shell_l[:nhs] + 1))
    P = torch.from_numpy(cl.P).cuda()
    K = torch.full((nh, cl.nbf), 7.0, dtype=torch.float64, device="cuda")
    st = hfx.build_K_periodic(p, nhs, P, K, o, stats=True)
    torch.cuda.synchronize()
    return K.cpu().numpy(), st


@pytest.mark.parametrize("omega", [0.0, hi.OMEGA_HSE])
@pytest.mark.parametrize("case", ["chain_sp", "cube_spd", "two_atoms_spd"])
def test_periodic_equals_oracle(case, omega):
    if case == "chain_sp":
        cl = hi.periodic_cluster(natom_cell=1, reach=(2, 0, 0), lmax=1, nprim_range=(1, 2))
    elif case == "cube_spd":
        cl = hi.periodic_cluster(natom_cell=1, reach=(1, 1, 1), lmax=2, nprim_range=(1, 2))
    else:
        cl = hi.periodic_cluster(natom_cell=2, cell_len=6.0, reach=(1, 1, 0), lmax=2, nprim_range=(1, 3), seed=8)
    tau = 1e-10
    _say("periodic", case, omega, cl.nshell, "shells", cl.nbf, "functions")
    Ko, cnt = oracle.build_K_periodic(cl, tau=tau, omega=omega)
    Kg, st = _gpu(cl, tau, omega, prim_tau=0.0)
    err = np.abs(Kg - Ko).max()
    _say("  max |dK|", err, "max |K|", np.abs(Ko).max(), "quartets", st["quartets"], cnt["quartets"])
    assert err <= 1e-10
    assert st["quartets"] == cnt["quartets"]
    assert list(st["class_quartets"]) == list(cnt["per_class"])
    assert st["prim_quartets"] == cnt["prim_quartets"]


def test_periodic_default_prim_skipping_and_home_only():
    """Default primitive skipping stays within the bar; a cluster of the home
    cell alone gives the molecular K."""
    cl = hi.periodic_cluster(natom_cell=2, cell_len=6.0, reach=(1, 0, 1), lmax=2, nprim_range=(2, 4), seed=9)
    Ko, _ = oracle.build_K_periodic(cl, tau=1e-10, omega=hi.OMEGA_HSE)
    Kg, _ = _gpu(cl, 1e-10, hi.OMEGA_HSE)
    assert np.abs(Kg - Ko).max() <= 1e-10
    one = hi.periodic_cluster(natom_cell=3, reach=(0, 0, 0), lmax=2, nprim_range=(1, 3))
    Kp, _ = _gpu(one, 1e-10, hi.OMEGA_HSE)
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    p = hfx.pairs_from_system(one, o)
    P = torch.from_numpy(one.P).cuda()
    Km = torch.empty_like(P)
    hfx.build_K(p, P, Km, o)
    torch.cuda.synchronize()
    assert np.abs(Kp - Km.cpu().numpy()).max() <= 1e-12


def test_periodic_rejects_bad_arguments():
    cl = hi.periodic_cluster(natom_cell=1, reach=(1, 0, 0), lmax=1, nprim_range=(1, 1))
    o = hfx.opts(tau=1e-10, omega=0.11)
    p = hfx.pairs_from_system(cl, o)
    P = torch.from_numpy(cl.P).cuda()
    K = torch.empty((4, cl.nbf), dtype=torch.float64, device="cuda")
    for nh in (0, cl.nshell + 1):
        with pytest.raises(hfx.HfxError) as e:
            hfx.build_K_periodic(p, nh, P, K, o)
        assert e.value.status == hfx.HFX_EINVAL
    with pytest.raises(hfx.HfxError) as e:
        hfx.build_K_periodic(p, 2, P, K, hfx.opts(tau=1e-10, omega=0.11, prec=hfx.PREC_MIXED))
    assert e.value.status == hfx.HFX_EUNSUPPORTED
