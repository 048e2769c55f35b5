"""ctypes binding of the FP64 CPU oracle (kzk_oracle.c) plus the adjoint-workload loss.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kzk_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP over independent lines)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("nt", ctypes.c_int), ("ny", ctypes.c_int),
        ("tau0", ctypes.c_double), ("Lt", ctypes.c_double),
        ("y0", ctypes.c_double), ("Ly", ctypes.c_double),
        ("x0", ctypes.c_double), ("h", ctypes.c_double),
        ("A", ctypes.c_double), ("eps", ctypes.c_double),
        ("lf_global", ctypes.c_int),
        ("Dbar", ctypes.POINTER(ctypes.c_double)),
        ("nl", ctypes.POINTER(ctypes.c_double)),
        ("nsteps_max", ctypes.c_int),
        ("force0", ctypes.POINTER(ctypes.c_double)),
        ("force1", ctypes.POINTER(ctypes.c_double)),
        ("scheme", ctypes.c_int),
        ("reg_eps", ctypes.c_double),
        ("vel", ctypes.c_int),
        ("vel_modes", ctypes.c_int),
        ("vel_phi", ctypes.POINTER(ctypes.c_double)),
        ("vel_theta", ctypes.POINTER(ctypes.c_double)),
        ("vel_lambda", ctypes.c_double),
        ("vel_sigma_u", ctypes.c_double),
        ("vel_c0", ctypes.c_double),
        ("vel_prof", ctypes.POINTER(ctypes.c_double)),
    ]


@contextlib.contextmanager
def using_library(path: str):
    """Run the functions of this module on another build of the oracle (the
    mutation checks of the test-suite load copies with planted mistakes)."""
    global _lib
    saved = _lib
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _load(_LIB)
    return _lib


def _load(path: str):
    """Load one build of the oracle and declare its functions."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_fft.argtypes = [dp, ctypes.c_int, ctypes.c_int]
    L.orc_fft2.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.orc_phi.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
    L.orc_symbol.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp]
    L.orc_weno_b.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, dp]
    L.orc_weno_b_adj.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, dp, dp, dp]
    L.orc_run.argtypes = [ctypes.POINTER(_Cfg), dp, ctypes.c_int, ctypes.c_int]
    L.orc_run.restype = ctypes.c_int
    L.orc_adjoint.argtypes = [ctypes.POINTER(_Cfg), dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.orc_adjoint.restype = ctypes.c_int
    L.orc_velocity.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_double, ctypes.c_double, dp]
    L.orc_eval_b.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_double, ctypes.c_double, dp, dp]
    L.orc_last_step_seconds.argtypes = []
    L.orc_last_step_seconds.restype = ctypes.c_double
    return L


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def fft(x: np.ndarray, sign: int = -1) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    lib().orc_fft(_dp(a.view(np.float64)), a.shape[0], sign)
    return a


def fft2(x: np.ndarray, sign: int = -1) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    ny, nt = a.shape
    lib().orc_fft2(_dp(a.view(np.float64)), ny, nt, sign)
    return a


def phi(k: int, z) -> np.ndarray:
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    out = np.empty_like(z)
    r, i = ctypes.c_double(), ctypes.c_double()
    for idx, v in enumerate(z.ravel()):
        lib().orc_phi(k, v.real, v.imag, ctypes.byref(r), ctypes.byref(i))
        out.ravel()[idx] = complex(r.value, i.value)
    return out


class Cfg:
    """Holds the ctypes struct and keeps its arrays alive."""

    def __init__(self, p, n_steps=None, lf_global=None, force0=None, force1=None):
        ns = p.n_steps if n_steps is None else n_steps
        self.Dbar = np.ascontiguousarray(p.D_step[:ns], dtype=np.float64)
        self.nl = np.ascontiguousarray(p.nl_node[:ns + 1], dtype=np.float64)
        if len(self.Dbar) < ns or len(self.nl) < ns + 1:
            raise ValueError("coefficient schedule shorter than n_steps")
        self.f0 = None if force0 is None else np.ascontiguousarray(force0, dtype=np.float64)
        self.f1 = None if force1 is None else np.ascontiguousarray(force1, dtype=np.float64)
        null = ctypes.POINTER(ctypes.c_double)()
        vel = int(getattr(p, "vel", 0))
        arr = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        self.vphi, self.vtheta = arr(getattr(p, "vel_phi", None)), arr(getattr(p, "vel_theta", None))
        self.vprof = arr(getattr(p, "vel_prof", None))
        ptr = lambda a: null if a is None else _dp(a)
        self.c = _Cfg(p.n_tau, p.n_y, p.tau0, p.L_tau, p.y0, p.L_y, p.x0, p.h, p.A, p.weno_eps,
                      int(p.lf_scope if lf_global is None else lf_global),
                      _dp(self.Dbar), _dp(self.nl), ns,
                      null if self.f0 is None else _dp(self.f0),
                      null if self.f1 is None else _dp(self.f1),
                      int(getattr(p, "scheme", 0)), float(getattr(p, "reg_eps", 0.0)),
                      vel, int(getattr(p, "vel_modes", 0)), ptr(self.vphi), ptr(self.vtheta),
                      float(getattr(p, "vel_lambda", 0.0)), float(getattr(p, "vel_sigma_u", 0.0)),
                      float(getattr(p, "vel_c0", 1.0)), ptr(self.vprof))


def symbol(p, m: int, n: int, Dbar: float) -> complex:
    c = Cfg(p, n_steps=0)
    r, i = ctypes.c_double(), ctypes.c_double()
    lib().orc_symbol(ctypes.byref(c.c), m, n, Dbar, ctypes.byref(r), ctypes.byref(i))
    return complex(r.value, i.value)


def velocity(p, x: float, y: float) -> np.ndarray:
    """(U_par, U_perp, d_y U_perp) of the problem's velocity field at (x, y)."""
    c = Cfg(p, n_steps=0)
    out = np.zeros(3)
    lib().orc_velocity(ctypes.byref(c.c), float(x), float(y), _dp(out))
    return out


def eval_b(p, x: float, nl: float, u: np.ndarray) -> np.ndarray:
    """b(x, u) on the whole field, as the stepper evaluates it."""
    c = Cfg(p, n_steps=0)
    u = np.ascontiguousarray(u, dtype=np.float64)
    b = np.empty_like(u)
    lib().orc_eval_b(ctypes.byref(c.c), float(x), float(nl), _dp(u), _dp(b))
    return b


def weno_b(u: np.ndarray, dtau: float, nl: float, alpha: float, eps: float = 1e-6) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    b = np.empty_like(u)
    lib().orc_weno_b(_dp(u), u.shape[0], dtau, nl, alpha, eps, _dp(b))
    return b


def weno_b_adj(u, dtau, nl, alpha, g, eps=1e-6):
    u = np.ascontiguousarray(u, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    ub = np.empty_like(u)
    ab = ctypes.c_double()
    lib().orc_weno_b_adj(_dp(u), u.shape[0], dtau, nl, alpha, eps, _dp(g), _dp(ub), ctypes.byref(ab))
    return ub, ab.value


def run(p, n_steps=None, first=0, u=None, lf_global=None, force0=None, force1=None) -> np.ndarray:
    """Advance p.u0 (or u) by n_steps ExpRK22 steps starting at step `first`."""
    ns = p.n_steps if n_steps is None else n_steps
    c = Cfg(p, n_steps=first + ns, lf_global=lf_global, force0=force0, force1=force1)
    a = np.ascontiguousarray(p.u0 if u is None else u, dtype=np.float64).copy()
    rc = lib().orc_run(ctypes.byref(c.c), _dp(a), first, ns)
    if rc != 0:
        raise RuntimeError("orc_run failed: %d" % rc)
    return a


def last_step_seconds() -> float:
    """Wall time of the step loop of the last run() (transforms excluded)."""
    return float(lib().orc_last_step_seconds())


def adjoint(p, lam_end: np.ndarray, n_steps=None, ckpt=50, u0=None, first=0, lf_global=None) -> np.ndarray:
    ns = p.n_steps if n_steps is None else n_steps
    c = Cfg(p, n_steps=first + ns, lf_global=lf_global)
    u = np.ascontiguousarray(p.u0 if u0 is None else u0, dtype=np.float64)
    lam = np.ascontiguousarray(lam_end, dtype=np.float64).copy()
    rc = lib().orc_adjoint(ctypes.byref(c.c), _dp(u), _dp(lam), first, ns, ckpt)
    if rc != 0:
        raise RuntimeError("orc_adjoint failed: %d" % rc)
    return lam


def window_mask(p, lo=-2.0, hi=2.0) -> np.ndarray:
    y = p.y()
    return (y >= lo) & (y < hi)


def loss_and_grad(p, u: np.ndarray, kappa=20.0, lo=-2.0, hi=2.0):
    """Ground-signature loss of the adjoint workload over the central window
    W = {y in [lo, hi)} x all tau:  L = (1/kappa) log(mean_W e^{kappa u}) + mean_W u^2.
    Returns (L, dL/du) with the analytic gradient."""
    w = window_mask(p, lo, hi)
    uw = u[w, :]
    nW = uw.size
    mx = uw.max()
    e = np.exp(kappa * (uw - mx))
    se = e.sum()
    L = mx + np.log(se / nW) / kappa + (uw * uw).sum() / nW
    g = np.zeros_like(u)
    g[w, :] = e / se + 2.0 * uw / nW
    return float(L), g
