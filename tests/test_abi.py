"""The C-ABI library loads and exports every function include/regc.h declares,
and the host-side validation rejects bad inputs before touching a GPU.  CPU only:
no compute call is made."""
import ctypes
import os
import re

import pytest

from paper_1908_11118_amd import regc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "regc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(regc_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert _declared() == sorted(regc.EXPORTS)


def test_library_exports_every_symbol():
    if not os.path.exists(regc.LIB_PATH):
        pytest.skip("libregc_hip.so not built")
    lib = ctypes.CDLL(regc.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_opts_and_errors_without_gpu():
    if not os.path.exists(regc.LIB_PATH):
        pytest.skip("libregc_hip.so not built")
    L = regc.lib()
    o = regc.Opts()
    L.regc_default_opts(ctypes.byref(o))
    assert o.seed == 1 and o.p_disp == 0.5 and o.p_ins == 0.25 and o.swap_every == 10
    assert L.regc_strerror(regc.ENOCONV).decode().startswith("reweighting")
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    assert L.regc_create(None, None, None, None, ctypes.byref(h)) == regc.EINVAL
    assert b"null" in L.regc_last_error()
    pot = regc.Potential(1, 1, 1, 1, 2.5, 0.5, 1, 0)
    sys_ = regc.System(0, None, 4.0, 4.0, 0.0, 8.0, 1.0, 10)   # box below 2 rcut
    t = (ctypes.c_double * 1)(1.0)
    g = regc.Grid(1, 1, t, t)
    assert L.regc_create(ctypes.byref(pot), ctypes.byref(sys_), ctypes.byref(g), ctypes.byref(o),
                         ctypes.byref(h)) == regc.EINVAL
    o.p_ins = 0.3                                                # unequal insertion/removal
    sys_.lx = sys_.ly = 6.0
    assert L.regc_create(ctypes.byref(pot), ctypes.byref(sys_), ctypes.byref(g), ctypes.byref(o),
                         ctypes.byref(h)) == regc.EINVAL
    L.regc_default_opts(ctypes.byref(o))
    mu_nan = (ctypes.c_double * 1)(float("nan"))                 # non-finite mu, then T
    g_bad = regc.Grid(1, 1, t, mu_nan)
    assert L.regc_create(ctypes.byref(pot), ctypes.byref(sys_), ctypes.byref(g_bad), ctypes.byref(o),
                         ctypes.byref(h)) == regc.EINVAL
    assert b"mu" in L.regc_last_error()
    t_inf = (ctypes.c_double * 1)(float("inf"))
    g_bad = regc.Grid(1, 1, t_inf, t)
    assert L.regc_create(ctypes.byref(pot), ctypes.byref(sys_), ctypes.byref(g_bad), ctypes.byref(o),
                         ctypes.byref(h)) == regc.EINVAL
    pot.mode = 2                                                 # site lattice: oracle only
    assert L.regc_create(ctypes.byref(pot), ctypes.byref(sys_), ctypes.byref(g), ctypes.byref(o),
                         ctypes.byref(h)) == regc.EUNSUPPORTED


def test_each_precision_has_its_own_kernel_symbols():
    """The FP64 and FP32 builds of the sweep kernel must not share symbol names,
    or one precision's launches run the other's code."""
    if not os.path.exists(regc.LIB_PATH):
        pytest.skip("libregc_hip.so not built")
    blob = open(regc.LIB_PATH, "rb").read()
    names = set(re.findall(rb"_ZN4regc4fp(?:32|64)12sweep_kernelILi[12]ELb[01]EEEvNS_9SweepArgsE", blob))
    assert len(names) == 8, sorted(names)
    assert not re.search(rb"_ZN4regc12sweep_kernel", blob)
