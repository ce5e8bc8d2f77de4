"""Batched persistent launch (device work queue + autotuner) and the
continuous-batching server: every system's K is the same alone, in a batch
and in the served mix (FP64 atomics only change the summation order, so the
bar is 1e-12 hartree), and matches the oracle on small systems."""

import os
import sys
import time

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


def _systems(n=5, seed=40):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        natom = int(rng.integers(2, 7))
        lmax = int(rng.integers(1, 3))
        out.append(hi.lattice_system(natom, seed=seed + i, lmax=lmax, nprim_range=(1, 3)))
    return out


def _solo(s, o):
    p = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    K = torch.empty_like(P)
    st = hfx.build_K(p, P, K, o, stats=True)
    torch.cuda.synchronize()
    return K.cpu().numpy(), st


@pytest.mark.parametrize("prec", [hfx.PREC_FP64, hfx.PREC_MIXED])
def test_batch_equals_solo_and_oracle(prec):
    systems = _systems()
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE, prec=prec)
    pairs = [hfx.pairs_from_system(s, o) for s in systems]
    Ps = [torch.from_numpy(s.P).cuda() for s in systems]
    Ks = [torch.empty_like(P) for P in Ps]
    _say("batch", [s.natom for s in systems], "prec", prec)
    st = hfx.build_K_batch(pairs, Ps, Ks, o, stats=True)
    torch.cuda.synchronize()
    nq = 0
    for s, K in zip(systems, Ks):
        Ksolo, sts = _solo(s, o)
        Kb = K.cpu().numpy()
        assert np.abs(Kb - Ksolo).max() <= 1e-12, np.abs(Kb - Ksolo).max()
        nq += sts["quartets"]
        if prec == hfx.PREC_FP64:
            Ko, _, _ = oracle.build_K(s, tau=1e-10, omega=hi.OMEGA_HSE)
            assert np.abs(Kb - Ko).max() <= 1e-10
    assert st["quartets"] == nq
    # a second call reuses the tuned parameters and the resident lists
    st2 = hfx.build_K_batch(pairs, Ps, Ks, o, stats=True)
    assert st2["quartets"] == nq


def test_batch_default_parameters_equal_tuned():
    """HFX_TUNE=0 runs the batch with the default launch parameters (no
    autotuning): the same K and quartet count as the tuned batch."""
    systems = _systems(n=4, seed=60)
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    pairs = [hfx.pairs_from_system(s, o) for s in systems]
    Ps = [torch.from_numpy(s.P).cuda() for s in systems]
    K1 = [torch.empty_like(P) for P in Ps]
    K2 = [torch.empty_like(P) for P in Ps]
    st1 = hfx.build_K_batch(pairs, Ps, K1, o, stats=True)
    os.environ["HFX_TUNE"] = "0"
    try:
        st2 = hfx.build_K_batch(pairs, Ps, K2, o, stats=True)
    finally:
        del os.environ["HFX_TUNE"]
    torch.cuda.synchronize()
    _say("batch tuned vs default parameters: quartets", st1["quartets"], st2["quartets"])
    assert st1["quartets"] == st2["quartets"]
    for a, b in zip(K1, K2):
        assert torch.abs(a - b).max().item() <= 1e-12


def test_batch_runs_large_systems_on_the_direct_kernels():
    """A system of at least 250 basis functions is built with the direct
    kernels inside the batch, the small ones through the persistent queue:
    every K equals its solo build, and the counts add up."""
    systems = _systems(n=3, seed=70) + [hi.lattice_system(24, seed=71, nprim_range=(1, 2))]
    assert systems[-1].nbf >= 250 and all(s.nbf < 250 for s in systems[:-1])
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    pairs = [hfx.pairs_from_system(s, o) for s in systems]
    Ps = [torch.from_numpy(s.P).cuda() for s in systems]
    Ks = [torch.empty_like(P) for P in Ps]
    st = hfx.build_K_batch(pairs, Ps, Ks, o, stats=True)
    torch.cuda.synchronize()
    nq = 0
    for s, K in zip(systems, Ks):
        Ksolo, sts = _solo(s, o)
        assert np.abs(K.cpu().numpy() - Ksolo).max() <= 1e-12
        nq += sts["quartets"]
    _say("batch with one direct system: quartets", st["quartets"], nq)
    assert st["quartets"] == nq


def test_batch_rejects_duplicate_handle():
    s = hi.sp8_cluster()
    o = hfx.opts(omega=0.11)
    p = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    K1, K2 = torch.empty_like(P), torch.empty_like(P)
    with pytest.raises(hfx.HfxError) as e:
        hfx.build_K_batch([p, p], [P, P], [K1, K2], o)
    assert e.value.status == hfx.HFX_EINVAL


def test_batch_empty():
    assert hfx.build_K_batch([], [], [], hfx.opts(), stats=True)["quartets"] == 0


def test_served_equals_solo_in_mix():
    """Requests of several systems, three SCF-like iterations each with a
    perturbed P, submitted together: four workers run them concurrently; each
    K equals the system's K built alone and the oracle's K for the same P."""
    systems = _systems(n=6, seed=50)
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    pairs = [hfx.pairs_from_system(s, o) for s in systems]
    srv = hfx.Server(hbm_budget_bytes=1 << 34, max_inflight=4)
    rng = np.random.default_rng(3)
    jobs = []
    for it in range(3):
        for i, s in enumerate(systems):
            Pn = hi.perturbed_density(s.P, rng)
            P = torch.from_numpy(Pn).cuda()
            K = torch.empty_like(P)
            torch.cuda.synchronize()
            t = srv.submit(pairs[i], P, K, o)
            jobs.append((i, Pn, P, K, t))
    done = {}
    t_end = time.time() + 120
    while len(done) < len(jobs) and time.time() < t_end:
        for (i, Pn, P, K, t) in jobs:
            if t in done:
                continue
            ok, st = srv.poll(t)
            if ok:
                done[t] = st
        time.sleep(0.01)
    assert len(done) == len(jobs)
    lat = sorted(st["latency_s"] for st in done.values())
    _say("served", len(jobs), "requests; p50 %.3f s p99 %.3f s" % (np.percentile(lat, 50), np.percentile(lat, 99)))
    for (i, Pn, P, K, t) in jobs:
        s = systems[i]
        Ps = torch.from_numpy(Pn).cuda()
        Kref = torch.empty_like(Ps)
        ps = hfx.pairs_from_system(s, o)
        hfx.build_K(ps, Ps, Kref, o)
        torch.cuda.synchronize()
        assert torch.abs(K - Kref).max().item() <= 1e-12
        Ko, _, _ = oracle.build_K(s, tau=1e-10, omega=hi.OMEGA_HSE, P=Pn)
        assert np.abs(K.cpu().numpy() - Ko).max() <= 1e-10
    with pytest.raises(hfx.HfxError) as e:
        srv.poll(jobs[0][4])  # already collected
    assert e.value.status == hfx.HFX_ENOTFOUND


def test_server_admission_and_errors():
    s = hi.sp8_cluster()
    o = hfx.opts(omega=0.11)
    p = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    K = torch.empty_like(P)
    small = hfx.Server(hbm_budget_bytes=1024, max_inflight=2)
    with pytest.raises(hfx.HfxError) as e:
        small.submit(p, P, K, o)
    assert e.value.status == hfx.HFX_ENOMEM
    with pytest.raises(hfx.HfxError) as e:
        small.poll(12345)
    assert e.value.status == hfx.HFX_ENOTFOUND
    # a budget that fits one request at a time still serves all of them
    one = hfx.Server(hbm_budget_bytes=p.device_bytes + 2 * 8 * s.nbf * s.nbf + 64, max_inflight=3)
    q = [hfx.pairs_from_system(s, o) for _ in range(3)]
    Ks = [torch.empty_like(P) for _ in range(3)]
    ts = [one.submit(q[i], P, Ks[i], o) for i in range(3)]
    t_end = time.time() + 60
    pend = set(ts)
    while pend and time.time() < t_end:
        for t in list(pend):
            if one.poll(t)[0]:
                pend.discard(t)
        time.sleep(0.01)
    assert not pend
    for i in range(1, 3):
        assert torch.abs(Ks[i] - Ks[0]).max().item() <= 1e-12


def test_server_queue_full_is_ebusy(monkeypatch):
    """A queue of capacity one behind one busy worker: a third quick
    submission finds it full (HFX_EBUSY); every accepted request completes
    with the solo K."""
    monkeypatch.setenv("HFX_SERVER_QUEUE", "1")
    s = hi.lattice_system(12, seed=61)
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    pairs = [hfx.pairs_from_system(s, o) for _ in range(6)]
    P = torch.from_numpy(s.P).cuda()
    Ks = [torch.empty_like(P) for _ in range(6)]
    torch.cuda.synchronize()
    srv = hfx.Server(hbm_budget_bytes=1 << 34, max_inflight=1)
    accepted, busy = [], 0
    for i in range(6):
        try:
            accepted.append((i, srv.submit(pairs[i], P, Ks[i], o)))
        except hfx.HfxError as e:
            assert e.status == hfx.HFX_EBUSY
            busy += 1
    _say("queue of one: accepted", len(accepted), "busy", busy)
    assert busy >= 1 and len(accepted) >= 1
    t_end = time.time() + 60
    pend = dict(accepted)
    while pend and time.time() < t_end:
        for i, t in list(pend.items()):
            if srv.poll(t)[0]:
                del pend[i]
        time.sleep(0.005)
    assert not pend
    Kref = torch.empty_like(P)
    hfx.build_K(hfx.pairs_from_system(s, o), P, Kref, o)
    torch.cuda.synchronize()
    for i, _ in accepted:
        assert torch.abs(Ks[i] - Kref).max().item() <= 1e-12
