"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: squared Schwarz factors (diagonal integrals) to 1e-13 of the largest,
raw integrals to 1e-12 of the quartet's Schwarz bound Q_IJ Q_KL, plain FP64 K
within 1e-10 hartree max-abs (the target accuracy of the FP64 build).
"""

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


def _gpu_K(s, tau, omega, stats=False, prim_tau=None):
    p = hfx.pairs_from_system(s, hfx.opts(tau=tau, omega=omega))
    P = torch.from_numpy(s.P).cuda()
    K = torch.empty_like(P)
    st = hfx.build_K(p, P, K, hfx.opts(tau=tau, omega=omega, prim_tau=prim_tau), stats=stats)
    torch.cuda.synchronize()
    return K.cpu().numpy(), st, p


def _pid(i, j):
    i, j = max(i, j), min(i, j)
    return i * (i + 1) // 2 + j


def _spd_small(seed=21, natom=3, nprim=(1, 3)):
    return hi.lattice_system(natom, seed=seed, nprim_range=nprim)


@pytest.mark.parametrize("omega", [0.0, hi.OMEGA_HSE])
def test_schwarz_factors(omega):
    for s in (hi.sp8_cluster(), _spd_small()):
        _say("schwarz", s.meta["name"], omega)
        p = hfx.pairs_from_system(s)
        q = hfx.schwarz_bounds(p, hfx.opts(omega=omega))
        qo = oracle.schwarz(s, omega=omega)
        # the bounds are square roots of diagonal integrals: compare those on an
        # absolute scale (a small diagonal value carries the rounding of its
        # larger contributions)
        err = np.abs(q ** 2 - qo ** 2).max()
        assert err <= 1e-13 * (qo ** 2).max(), err


@pytest.mark.parametrize("omega", [0.0, hi.OMEGA_HSE])
def test_raw_integrals_every_class(omega):
    """Every one of the 21 classes, both orders inside pairs and across."""
    s = _spd_small(seed=22, natom=2, nprim=(2, 3))
    p = hfx.pairs_from_system(s)
    rng = np.random.default_rng(5)
    quartets = []
    for I in range(s.nshell):
        for J in range(s.nshell):
            for K in range(s.nshell):
                for L in range(s.nshell):
                    if rng.random() < 0.02:
                        quartets.append((I, J, K, L))
    _say("eval", len(quartets), "quartets")
    got = hfx.eval_quartets(p, hfx.opts(omega=omega), quartets, s.shell_l)
    Q = oracle.schwarz(s, omega=omega)
    seen = set()
    for q, g in zip(quartets, got):
        ref = oracle.shell_quartet(s, *q, omega=omega)
        # rounding scale of a quartet: its Schwarz bound Q_IJ Q_KL
        bound = Q[_pid(q[0], q[1])] * Q[_pid(q[2], q[3])]
        assert np.abs(g - ref).max() <= 1e-12 * bound, (q, np.abs(g - ref).max(), bound)
        ls = sorted([tuple(sorted((s.shell_l[q[0]], s.shell_l[q[1]]), reverse=True)),
                     tuple(sorted((s.shell_l[q[2]], s.shell_l[q[3]]), reverse=True))], reverse=True)
        seen.add(tuple(ls))
    assert len(seen) == 21, len(seen)


@pytest.mark.parametrize("prim_tau", [0.0, None])
@pytest.mark.parametrize("omega", [0.0, hi.OMEGA_HSE])
def test_K_sp8_cluster(omega, prim_tau):
    """prim_tau = 0: every primitive quartet (same counts as the oracle);
    default: primitive quartets with bound below 1e-3 min(tau, 1e-10) skipped."""
    s = hi.sp8_cluster()
    _say("K sp8_cluster", omega, prim_tau)
    Ko, _, cnt = oracle.build_K(s, tau=1e-10, omega=omega)
    Kg, st, _ = _gpu_K(s, 1e-10, omega, stats=True, prim_tau=prim_tau)
    _say("  max |dK|", np.abs(Kg - Ko).max(), "prim quartets", st["prim_quartets"], "of", cnt["prim_quartets"])
    assert np.abs(Kg - Ko).max() <= 1e-10
    assert np.abs(Kg - Kg.T).max() == 0.0
    assert st["quartets"] == cnt["quartets"]
    if prim_tau == 0.0:
        assert st["prim_quartets"] == cnt["prim_quartets"]
    else:
        assert st["prim_quartets"] <= cnt["prim_quartets"]
    assert abs(np.trace(s.P @ Kg) - np.trace(s.P @ Ko)) <= 1e-10 * abs(np.trace(s.P @ Ko))


@pytest.mark.parametrize("prim_tau", [0.0, None])
@pytest.mark.parametrize("omega", [0.0, hi.OMEGA_HSE])
@pytest.mark.parametrize("tau", [0.0, 1e-10, 1e-6])
def test_K_dzp_small(omega, tau, prim_tau):
    """s, p and d shells; ket ranges longer than one 64-lane chunk with a
    ragged tail; tau = 0 (every quartet), tight and loose screening; with
    and without primitive-quartet skipping."""
    s = _spd_small(seed=23, natom=8, nprim=(1, 3))
    _say("K dzp8", omega, tau, prim_tau)
    Ko, _, cnt = oracle.build_K(s, tau=tau, omega=omega)
    Kg, st, _ = _gpu_K(s, tau, omega, stats=True, prim_tau=prim_tau)
    _say("  max |dK|", np.abs(Kg - Ko).max())
    assert np.abs(Kg - Ko).max() <= 1e-10, np.abs(Kg - Ko).max()
    assert st["quartets"] == cnt["quartets"]
    assert list(st["class_quartets"]) == list(cnt["per_class"])


def test_prim_skipping_error_dzp_full_contraction():
    """3-6 primitives per shell (the workload's contraction): the primitive
    quartets skipped at the default threshold (1e-13) change K by at most
    a fifth of the 1e-10 bar."""
    s = hi.lattice_system(6, seed=31)
    Ko, _, cnt = oracle.build_K(s, tau=1e-10, omega=hi.OMEGA_HSE)
    Kg, st, _ = _gpu_K(s, 1e-10, hi.OMEGA_HSE, stats=True)
    err = np.abs(Kg - Ko).max()
    _say("dzp6 full contraction: max |dK|", err, "prim", st["prim_quartets"], "of", cnt["prim_quartets"])
    assert err <= 2e-11
    assert st["prim_quartets"] < cnt["prim_quartets"]


def test_K_degenerate_single_shell_and_s_only():
    # one atom with one s shell: the only quartet is (II|II), degeneracy 1/8
    s = hi.tiny_sp_cluster(seed=3, natom=1, ls=(0,), nprim=2)
    Ko, _, _ = oracle.build_K(s, tau=0.0, omega=0.11)
    Kg, _, _ = _gpu_K(s, 0.0, 0.11)
    assert np.abs(Kg - Ko).max() <= 1e-13
    # s-only cluster, every primitive quartet evaluated (degeneracy factors
    # checked at rounding level)
    s = hi.tiny_sp_cluster(seed=4, natom=6, ls=(0,), nprim=3)
    Ko, _, _ = oracle.build_K(s, tau=1e-10, omega=0.0)
    Kg, _, _ = _gpu_K(s, 1e-10, 0.0, prim_tau=0.0)
    assert np.abs(Kg - Ko).max() <= 1e-12


def test_K_everything_screened_is_zero():
    s = hi.sp8_cluster()
    Kg, st, _ = _gpu_K(s, 1e6, 0.0, stats=True)
    assert st["quartets"] == 0
    assert not Kg.any()


def test_K_asymmetric_P_rejected():
    s = hi.sp8_cluster()
    p = hfx.pairs_from_system(s)
    P = torch.from_numpy(s.P).cuda()
    P[0, 1] += 1e-3
    K = torch.empty_like(P)
    with pytest.raises(hfx.HfxError) as e:
        hfx.build_K(p, P, K, hfx.opts())
    assert e.value.status == hfx.HFX_EASYM


def test_K_leading_dimension():
    s = hi.sp8_cluster()
    n = s.nbf
    big = torch.zeros((n, n + 7), dtype=torch.float64, device="cuda")
    big[:, :n] = torch.from_numpy(s.P).cuda()
    Kb = torch.full((n, n + 7), 7.0, dtype=torch.float64, device="cuda")
    p = hfx.pairs_from_system(s)
    hfx.build_K(p, big[:, :n], Kb[:, :n], hfx.opts(omega=0.11))
    torch.cuda.synchronize()
    Ko, _, _ = oracle.build_K(s, tau=1e-10, omega=0.11)
    Kg = Kb.cpu().numpy()
    assert np.abs(Kg[:, :n] - Ko).max() <= 1e-10
    assert (Kg[:, n:] == 7.0).all()


def test_repeat_build_reuses_lists_and_is_stable():
    s = _spd_small(seed=24, natom=5, nprim=(2, 3))
    p = hfx.pairs_from_system(s)
    P = torch.from_numpy(s.P).cuda()
    K1 = torch.empty_like(P)
    K2 = torch.empty_like(P)
    o = hfx.opts(tau=1e-10, omega=0.11)
    hfx.build_K(p, P, K1, o)
    hfx.build_K(p, P * 2.0, K2, o)
    torch.cuda.synchronize()
    assert torch.allclose(K2, 2.0 * K1, rtol=1e-12, atol=1e-14)


def _class_counts(s, Q, tau):
    """Screened unique quartets per (bra class, ket class), counted with numpy
    from the Schwarz factors alone: pair classes by (max l, min l), bra class >=
    ket class, and within one class only the lower triangle of pair pairs."""
    n = s.nshell
    I = np.repeat(np.arange(n), np.arange(1, n + 1))
    J = np.concatenate([np.arange(i + 1) for i in range(n)])
    la = np.maximum(s.shell_l[I], s.shell_l[J])
    lb = np.minimum(s.shell_l[I], s.shell_l[J])
    cls = la * (la + 1) // 2 + lb
    out = np.zeros(21, dtype=np.int64)
    for cb in range(6):
        for ck in range(cb + 1):
            qb, qk = Q[cls == cb], np.sort(Q[cls == ck])
            cnt = sum(len(qk) - np.searchsorted(qk, tau / q, side="left") for q in qb if q > 0)
            if cb == ck:
                cnt = (cnt + int((qb * qb >= tau).sum())) // 2
            out[cb * (cb + 1) // 2 + ck] = cnt
    return out


@pytest.mark.parametrize("prec", [hfx.PREC_FP64, hfx.PREC_MIXED])
def test_segmented_launch(monkeypatch, prec):
    """A class grid above the per-launch block limit runs as several launches,
    each starting at its own logical block.  Forcing a limit of one XCD span
    cuts every class of a 12-atom lattice into many segments: every screened
    quartet is still evaluated once (per-class counts equal an independent
    count) and K equals the single-launch K."""
    s = hi.lattice_system(12, seed=31, nprim_range=(1, 3))
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE, prec=prec)
    p = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    K1, K2 = torch.empty_like(P), torch.empty_like(P)
    st1 = hfx.build_K(p, P, K1, o, stats=True)
    torch.cuda.synchronize()
    monkeypatch.setenv("HFX_MAX_BLOCKS", "1")
    _say("segmented launch, 12 atoms, prec", prec)
    st2 = hfx.build_K(p, P, K2, o, stats=True)
    torch.cuda.synchronize()
    monkeypatch.delenv("HFX_MAX_BLOCKS")
    want = _class_counts(s, hfx.schwarz_bounds(p, o), 1e-10)
    assert list(st1["class_quartets"]) == list(want)
    assert list(st2["class_quartets"]) == list(want)
    assert st2["quartets_fp32"] == st1["quartets_fp32"]
    assert torch.abs(K2 - K1).max().item() <= 1e-12


def test_full_size_dzp256_lattice_sampled():
    """configs-1 system at full size (1280 shells): all 819,840 Schwarz factors
    on the GPU; a sample of them and of raw quartet integrals (every class)
    against the oracle one by one."""
    s = hi.dzp256_lattice()
    _say("dzp256_lattice pairs")
    p = hfx.pairs_from_system(s)
    q = hfx.schwarz_bounds(p, hfx.opts(omega=hi.OMEGA_HSE))
    assert q.shape == (1280 * 1281 // 2,)
    rng = np.random.default_rng(9)
    idx = rng.choice(len(q), 300, replace=False)
    for pid in idx:
        I = int((np.sqrt(8 * pid + 1) - 1) // 2)
        while I * (I + 1) // 2 > pid:
            I -= 1
        while (I + 1) * (I + 2) // 2 <= pid:
            I += 1
        J = pid - I * (I + 1) // 2
        blk = oracle.shell_quartet(s, I, J, I, J, omega=hi.OMEGA_HSE)
        ni, nj = blk.shape[:2]
        qo = np.sqrt(max(blk[i, j, i, j] for i in range(ni) for j in range(nj)))
        assert abs(q[pid] ** 2 - qo ** 2) <= 1e-13 * max(qo ** 2, 1e-3)
    quartets = rng.integers(0, s.nshell, size=(400, 4))
    got = hfx.eval_quartets(p, hfx.opts(omega=hi.OMEGA_HSE), quartets, s.shell_l)
    for qq, g in zip(quartets, got):
        ref = oracle.shell_quartet(s, *qq, omega=hi.OMEGA_HSE)
        bound = q[_pid(qq[0], qq[1])] * q[_pid(qq[2], qq[3])]
        assert np.abs(g - ref).max() <= 1e-12 * bound + 1e-300


def test_full_size_bench_shard_properties():
    """The bench's launch configuration (256-atom system, shard 0 of 64, erfc,
    tau = 1e-10): K is linear in P (K(P + 2E) = K(P) + 2 K(E) for a
    symmetric E, so no P-dependent work is skipped and no update is lost or
    doubled between runs), exactly symmetric, and zero for P = 0."""
    s = hi.dzp256_lattice()
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    p = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    rng = np.random.default_rng(77)
    E = rng.standard_normal(s.P.shape) * (s.P != 0)
    E = torch.from_numpy(0.5 * (E + E.T)).cuda()
    Ks = []
    for X in (P, E, P + 2.0 * E):
        _say("bench shard build, 256 atoms, shard 0/64")
        K = torch.empty_like(P)
        hfx.build_K_shard(p, X.contiguous(), K, o, 0, 64)
        torch.cuda.synchronize()
        Ks.append(K)
    scale = max(torch.abs(Ks[0]).max().item(), torch.abs(Ks[1]).max().item())
    assert torch.abs(Ks[2] - Ks[0] - 2.0 * Ks[1]).max().item() <= 1e-12 * scale
    for K in Ks:
        assert torch.equal(K, K.T)
    Z = torch.zeros_like(P)
    K0 = torch.empty_like(P)
    hfx.build_K_shard(p, Z, K0, o, 0, 64)
    torch.cuda.synchronize()
    assert torch.count_nonzero(K0).item() == 0
