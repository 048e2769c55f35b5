"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every function declared in include/kzk.h, and argument errors are rejected
before anything touches the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kzk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kzk_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["kzk_create", "kzk_step", "kzk_adjoint", "kzk_poll", "kzk_destroy", "kzk_inst_offset",
              "kzk_status_str"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2103_06080_amd import kzk
    L = kzk.lib()
    for n in declared_functions():
        assert hasattr(L, n), n
    assert sorted(kzk.EXPORTS) == declared_functions()


def test_status_strings():
    from paper_2103_06080_amd import kzk
    L = kzk.lib()
    for code in range(8):
        assert L.kzk_status_str(code)


def _params(**kw):
    from paper_2103_06080_amd import kzk
    base = dict(n_tau=64, n_y=32, tau0=-4.0, L_tau=8.0, y0=-8.0, L_y=16.0, x0=0.0, h=1e-3, dtype=1,
                D=0.05, A=0.0, nl=1.0, D_step=None, nl_node=None, n_steps_max=0, lf_scope=0,
                weno_eps=1e-6, cfl_max=1.0, scheme=0, reg_eps=0.0, vel=0, state_fp64=0)
    base.update(kw)
    null = ctypes.POINTER(ctypes.c_double)()
    return kzk.Params(base["n_tau"], base["n_y"], base["tau0"], base["L_tau"], base["y0"], base["L_y"],
                      base["x0"], base["h"], base["dtype"], base["D"], base["A"], base["nl"], null, null,
                      base["n_steps_max"], base["lf_scope"], base["weno_eps"], base["cfl_max"],
                      base["scheme"], base["reg_eps"], base["vel"], 0, null, null, 0.0, 0.0, 0.0,
                      base["state_fp64"])


@pytest.mark.parametrize("kw,code", [
    (dict(n_tau=48), 2), (dict(n_tau=16), 2), (dict(n_tau=16384), 2), (dict(n_y=8), 2), (dict(n_y=16384), 2),
    (dict(n_tau=112), 2), (dict(n_tau=14336), 2), (dict(n_tau=96), 2), (dict(n_tau=480), 2), (dict(n_y=448), 2),
    (dict(h=0.0), 1), (dict(h=-1.0), 1), (dict(L_tau=0.0), 1), (dict(dtype=3), 1), (dict(A=-1.0), 1),
    (dict(weno_eps=0.0), 1), (dict(lf_scope=1), 1), (dict(cfl_max=-1.0), 1),
    (dict(scheme=2), 1), (dict(scheme=-1), 1), (dict(reg_eps=-1e-16), 1), (dict(reg_eps=float("nan")), 1),
    (dict(vel=2), 1), (dict(vel=1), 1), (dict(state_fp64=2), 1), (dict(state_fp64=1, dtype=0, reg_eps=1e-7), 1),
])
def test_create_rejects_bad_parameters_before_device_work(kw, code):
    from paper_2103_06080_amd import kzk
    L = kzk.lib()
    p = _params(**kw)
    h = ctypes.c_void_p()
    assert L.kzk_create(ctypes.byref(p), 1, None, ctypes.byref(h)) == code
    assert not h.value


def test_create_rejects_a_7_2k_plan_with_two_tau_lengths():
    """n_tau = 7 * 2^k: every solve of the plan has that n_tau (checked
    before any device work)."""
    from paper_2103_06080_amd import kzk
    L = kzk.lib()
    for a, b in ((448, 512), (512, 448), (448, 896)):
        ps = (kzk.Params * 2)(_params(n_tau=a), _params(n_tau=b))
        h = ctypes.c_void_p()
        assert L.kzk_create(ps, 2, None, ctypes.byref(h)) == 2, (a, b)
        assert not h.value


def test_null_arguments_rejected():
    from paper_2103_06080_amd import kzk
    L = kzk.lib()
    h = ctypes.c_void_p()
    assert L.kzk_create(None, 1, None, ctypes.byref(h)) == 1
    p = _params()
    assert L.kzk_create(ctypes.byref(p), 0, None, ctypes.byref(h)) == 1
    assert L.kzk_step(None, None, 0, 1) == 1
    assert L.kzk_poll(None) == 1
    assert L.kzk_adjoint(None, None, None, 0, 1, 1, None) == 1
    assert L.kzk_inst_offset(None, 0) == ctypes.c_size_t(-1).value
