"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the header declares, and rejects invalid input before any
device work."""

import ctypes
import os
import re

import numpy as np
import pytest

import hfx_inputs as hi
import paper_2009_03559_amd as hfx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hfx.h")).read()
    return sorted(set(re.findall(r"\b(hfx_[A-Za-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert sorted(hfx.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    L = hfx.lib()
    for name in _declared():
        assert hasattr(L, name), name


def _sys_args(s):
    return (s.xyz, s.shell_atom, s.shell_l, s.shell_nprim, s.shell_off, s.exps, s.coefs)


@pytest.mark.parametrize("mutate,status", [
    (lambda s: s.shell_l.__setitem__(0, 3), hfx.HFX_EUNSUPPORTED),
    (lambda s: s.shell_l.__setitem__(0, -1), hfx.HFX_EINVAL),
    (lambda s: s.exps.__setitem__(0, 0.0), hfx.HFX_EINVAL),
    (lambda s: s.exps.__setitem__(1, -2.0), hfx.HFX_EINVAL),
    (lambda s: s.exps.__setitem__(2, float("nan")), hfx.HFX_EINVAL),
    (lambda s: s.shell_atom.__setitem__(0, 99), hfx.HFX_EINVAL),
    (lambda s: s.shell_nprim.__setitem__(0, 0), hfx.HFX_EINVAL),
    (lambda s: s.shell_nprim.__setitem__(0, 17), hfx.HFX_EUNSUPPORTED),
])
def test_invalid_basis_rejected_on_host(mutate, status):
    s = hi.sp8_cluster()
    mutate(s)
    with pytest.raises(hfx.HfxError) as e:
        hfx.build_shell_pairs(*_sys_args(s), o=hfx.opts(), stream=0)
    assert e.value.status == status


def test_too_many_functions_rejected_on_host():
    """n_bf above HFX_MAX_NBF (65535): the n_bf^2 element kernels would pass
    the 32-bit work-item count of one dispatch."""
    natom = 13108  # one d shell each: 65540 functions
    xyz = np.zeros((natom, 3))
    xyz[:, 0] = 4.0 * np.arange(natom)
    atom = np.arange(natom, dtype=np.int32)
    ls = np.full(natom, 2, dtype=np.int32)
    npr = np.ones(natom, dtype=np.int32)
    off = np.arange(natom, dtype=np.int32)
    ex = np.ones(natom)
    with pytest.raises(hfx.HfxError) as e:
        hfx.build_shell_pairs(xyz, atom, ls, npr, off, ex, np.ones(natom), o=hfx.opts(), stream=0)
    assert e.value.status == hfx.HFX_EUNSUPPORTED


@pytest.mark.parametrize("kw,status", [
    (dict(tau=-1.0), hfx.HFX_EINVAL),
    (dict(omega=-0.1, op=hfx.OP_ERFC), hfx.HFX_EINVAL),
    (dict(prec=7), hfx.HFX_EINVAL),
    (dict(prim_tau=-1.0), hfx.HFX_EINVAL),
    (dict(flags=6), hfx.HFX_EINVAL),
])
def test_invalid_options_rejected_on_host(kw, status):
    s = hi.sp8_cluster()
    flags = kw.pop("flags", None)
    o = hfx.opts(**kw)
    if flags is not None:
        o.flags = flags
    with pytest.raises(hfx.HfxError) as e:
        hfx.build_shell_pairs(*_sys_args(s), o=o, stream=0)
    assert e.value.status == status


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(hfx, "_lib", None)
    monkeypatch.setattr(hfx, "LIB_PATH", "/nonexistent/libhfx.so")
    with pytest.raises(hfx.HfxError):
        hfx.lib()
