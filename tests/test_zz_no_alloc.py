"""The exchange build without device allocation (hfx_build_K_noalloc, called
through the C ABI) against hfx_build_K on the same handle and inputs: equal K
within 1e-12 hartree (FP64 atomics only change the summation order) and equal
quartet counts, on two calls in a row, the second with a smaller system; FP64
and mixed precision; an unprepared handle is refused without allocating."""

import sys

import numpy as np
import pytest

import hfx_inputs as hi
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


def _prepared(s, o):
    p = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    K = torch.empty_like(P)
    st = hfx.build_K(p, P, K, o, stats=True)
    torch.cuda.synchronize()
    return p, P, K, st


@pytest.mark.parametrize("prec", [hfx.PREC_FP64, hfx.PREC_MIXED])
def test_noalloc_equals_build_K_two_calls(prec):
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE, prec=prec)
    big = hi.lattice_system(12, seed=71)
    small = hi.lattice_system(5, seed=72)
    for s in (big, small):  # second call: a smaller input
        _say("no-alloc build", s.natom, "atoms, prec", prec)
        p, P, Kref, stref = _prepared(s, o)
        K = torch.full_like(P, 3.0)
        st = hfx.build_K_noalloc(p, P, K, o, stats=True)
        torch.cuda.synchronize()
        err = torch.abs(K - Kref).max().item()
        _say("  max |K_noalloc - K| =", err, "quartets", st["quartets"])
        assert err <= 1e-12
        assert st["quartets"] == stref["quartets"]
        assert st["quartets_fp32"] == stref["quartets_fp32"]
        assert st["class_quartets"] == stref["class_quartets"]
        # without statistics (no counters touched)
        K2 = torch.full_like(P, -1.0)
        hfx.build_K_noalloc(p, P, K2, o)
        torch.cuda.synchronize()
        assert torch.abs(K2 - Kref).max().item() <= 1e-12


def test_noalloc_refuses_unprepared_handle():
    s = hi.sp8_cluster()
    o = hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE)
    p = hfx.pairs_from_system(s, o)
    P = torch.from_numpy(s.P).cuda()
    K = torch.empty_like(P)
    with pytest.raises(hfx.HfxError) as e:
        hfx.build_K_noalloc(p, P, K, o)
    assert e.value.status == hfx.HFX_EINVAL
    hfx.build_K(p, P, K, o)
    # another tau needs other lists: refused as well
    with pytest.raises(hfx.HfxError) as e:
        hfx.build_K_noalloc(p, P, K, hfx.opts(tau=1e-8, omega=hi.OMEGA_HSE))
    assert e.value.status == hfx.HFX_EINVAL
    # mixed precision before any mixed build: no FP32 records yet
    with pytest.raises(hfx.HfxError) as e:
        hfx.build_K_noalloc(p, P, K, hfx.opts(tau=1e-10, omega=hi.OMEGA_HSE, prec=hfx.PREC_MIXED))
    assert e.value.status == hfx.HFX_EINVAL
    Kn = torch.empty_like(P)
    hfx.build_K_noalloc(p, P, Kn, o)
    torch.cuda.synchronize()
    assert torch.abs(Kn - K).max().item() <= 1e-12
