"""Thin ctypes binding of libkzk (include/kzk.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libkzk.so; PyTorch only
provides device memory and the current stream.  There is no fallback: if the
library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkzk.so")

KZK_F32, KZK_F64 = 0, 1
STATUS = {0: "KZK_OK", 1: "KZK_ERR_ARG", 2: "KZK_ERR_SIZE", 3: "KZK_ERR_OOM", 4: "KZK_ERR_DEVICE",
          5: "KZK_ERR_CFL", 6: "KZK_ERR_NONFINITE", 7: "KZK_ERR_STATE"}

EXPORTS = ["kzk_create", "kzk_step", "kzk_adjoint", "kzk_poll", "kzk_inst_offset", "kzk_set_stream",
           "kzk_set_graph", "kzk_set_y_threads", "kzk_get_y_threads", "kzk_destroy", "kzk_status_str",
           "kzk_eval_b", "kzk_tau_forward", "kzk_tau_inverse", "kzk_profile_enable", "kzk_profile_read",
           "kzk_read_tables", "kzk_autotune", "kzk_step_noalloc", "kzk_set_tau_threads",
           "kzk_get_tau_threads", "kzk_set_tau_fft_radix", "kzk_get_tau_fft_radix"]
KINDS = ["tau_pass", "y_pass1", "y_pass2", "tables", "tau_transform", "adj_tau_pass", "adj_y_pass", "transport"]


class KZKError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s failed: %s (%d)" % (what, STATUS.get(code, "?"), code))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("n_tau", ctypes.c_int32), ("n_y", ctypes.c_int32),
        ("tau0", ctypes.c_double), ("L_tau", ctypes.c_double),
        ("y0", ctypes.c_double), ("L_y", ctypes.c_double),
        ("x0", ctypes.c_double), ("h", ctypes.c_double),
        ("dtype", ctypes.c_int32),
        ("D", ctypes.c_double), ("A", ctypes.c_double), ("nl", ctypes.c_double),
        ("D_step", ctypes.POINTER(ctypes.c_double)),
        ("nl_node", ctypes.POINTER(ctypes.c_double)),
        ("n_steps_max", ctypes.c_int32),
        ("lf_scope", ctypes.c_int32),
        ("weno_eps", ctypes.c_double),
        ("cfl_max", ctypes.c_double),
        ("scheme", ctypes.c_int32),
        ("reg_eps", ctypes.c_double),
        ("vel", ctypes.c_int32),
        ("vel_modes", ctypes.c_int32),
        ("vel_phi", ctypes.POINTER(ctypes.c_double)),
        ("vel_theta", ctypes.POINTER(ctypes.c_double)),
        ("vel_lambda", ctypes.c_double),
        ("vel_sigma_u", ctypes.c_double),
        ("vel_c0", ctypes.c_double),
        ("state_fp64", ctypes.c_int32),
    ]


_lib = None


def lib():
    """Load libkzk.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libkzk.so is not built (run __graft_entry__.build()): %s" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        L.kzk_create.argtypes = [ctypes.POINTER(Params), i32, vp, ctypes.POINTER(vp)]
        L.kzk_step.argtypes = [vp, vp, i32, i32]
        L.kzk_adjoint.argtypes = [vp, vp, vp, i32, i32, i32, vp]
        L.kzk_poll.argtypes = [vp]
        L.kzk_inst_offset.argtypes = [vp, i32]
        L.kzk_inst_offset.restype = ctypes.c_size_t
        L.kzk_set_stream.argtypes = [vp, vp]
        L.kzk_set_graph.argtypes = [vp, i32]
        L.kzk_set_y_threads.argtypes = [vp, i32]
        L.kzk_get_y_threads.argtypes = [vp]
        L.kzk_get_y_threads.restype = i32
        L.kzk_destroy.argtypes = [vp]
        L.kzk_destroy.restype = None
        L.kzk_status_str.argtypes = [i32]
        L.kzk_status_str.restype = ctypes.c_char_p
        L.kzk_eval_b.argtypes = [vp, vp, i32, vp]
        L.kzk_tau_forward.argtypes = [vp, vp, vp]
        L.kzk_tau_inverse.argtypes = [vp, vp, vp]
        L.kzk_profile_enable.argtypes = [vp, i32]
        L.kzk_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32), i32]
        L.kzk_read_tables.argtypes = [vp, i32, vp]
        L.kzk_autotune.argtypes = [vp, vp, i32]
        L.kzk_autotune.restype = i32
        L.kzk_step_noalloc.argtypes = [ctypes.POINTER(Params), i32, vp, vp, i32, i32]
        L.kzk_set_tau_threads.argtypes = [vp, i32]
        L.kzk_get_tau_threads.argtypes = [vp]
        L.kzk_get_tau_threads.restype = i32
        L.kzk_set_tau_fft_radix.argtypes = [vp, i32]
        L.kzk_get_tau_fft_radix.argtypes = [vp]
        L.kzk_get_tau_fft_radix.restype = i32
        for name in EXPORTS:
            getattr(L, name)
        _lib = L
    return _lib


def _check(code: int, what: str):
    if code != 0:
        raise KZKError(code, what)


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def make_params(p, dtype: int, cfl_max: float = 1.0, keep: Optional[list] = None, state_fp64: bool = False) -> Params:
    """kzk_params from an inputs.Problem (schedules only for x-dependent coefficients)."""
    null = ctypes.POINTER(ctypes.c_double)()
    D_ptr, nl_ptr, nmax = null, null, 0
    if p.D_const is None or p.nl_const is None:
        D = np.ascontiguousarray(p.D_step, dtype=np.float64)
        nl = np.ascontiguousarray(p.nl_node, dtype=np.float64)
        if keep is not None:
            keep += [D, nl]
        D_ptr = D.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        nl_ptr = nl.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        nmax = len(D)
    vel = int(getattr(p, "vel", 0))
    vphi = vtheta = null
    if vel:
        if vel != 1:
            raise ValueError("the library takes vel = 0 or 1")
        a = np.ascontiguousarray(p.vel_phi, dtype=np.float64)
        b = np.ascontiguousarray(p.vel_theta, dtype=np.float64)
        D = np.ascontiguousarray(p.D_step, dtype=np.float64)
        nl = np.ascontiguousarray(p.nl_node, dtype=np.float64)
        if keep is not None:
            keep += [a, b, D, nl]
        vphi = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        vtheta = b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        # the field is tabulated at the nodes 0 .. n_steps_max; constant
        # coefficients still go without schedules (multiplier tables built once)
        nmax = max(nmax, len(D))
    return Params(p.n_tau, p.n_y, p.tau0, p.L_tau, p.y0, p.L_y, p.x0, p.h, dtype,
                  float(p.D_const if p.D_const is not None else 0.0), p.A,
                  float(p.nl_const if p.nl_const is not None else 0.0),
                  D_ptr, nl_ptr, nmax, p.lf_scope, p.weno_eps, cfl_max,
                  int(getattr(p, "scheme", 0)), float(getattr(p, "reg_eps", 0.0)),
                  vel, int(getattr(p, "vel_modes", 0)), vphi, vtheta,
                  float(getattr(p, "vel_lambda", 0.0)), float(getattr(p, "vel_sigma_u", 0.0)),
                  float(getattr(p, "vel_c0", 0.0)), 1 if state_fp64 else 0)


def step_noalloc(problems, u, first: int = 0, n_steps: int = 1, dtype: str = "f64", stream=None,
                 cfl_max: float = 1.0) -> int:
    """kzk_step_noalloc: march the packed field u (laid out as a Plan of the
    same problems packs it) without any device allocation; returns the status
    code (0 = ok; synchronises)."""
    if not isinstance(problems, (list, tuple)):
        problems = [problems]
    dt = KZK_F32 if dtype in ("f32", "float32") else KZK_F64
    keep: list = []
    arr = (Params * len(problems))(*[make_params(p, dt, cfl_max, keep) for p in problems])
    return lib().kzk_step_noalloc(arr, len(problems), ctypes.c_void_p(_stream_handle(stream)),
                                  ctypes.c_void_p(u.data_ptr()), int(first), int(n_steps))


class Plan:
    """A kzk_plan for one or several solves (uneven grids allowed).

    stream: the torch stream the plan enqueues on (default: the current
    stream).  graph=True replays marches as HIP graphs, which needs a stream
    other than the legacy default stream (kzk_step raises KZK_ERR_STATE
    there)."""

    def __init__(self, problems, dtype: str = "f64", stream=None, cfl_max: float = 1.0,
                 y_threads: Optional[int] = None, graph: bool = False, tau_threads: Optional[int] = None,
                 state_fp64: bool = False, tau_fft_radix: Optional[int] = None):
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        self.dtype = KZK_F32 if dtype in ("f32", "float32") else KZK_F64
        torch = _torch()
        self.tdtype = torch.float32 if self.dtype == KZK_F32 else torch.float64
        keep: list = []
        arr = (Params * len(problems))(*[make_params(p, self.dtype, cfl_max, keep, state_fp64) for p in problems])
        h = ctypes.c_void_p()
        _check(lib().kzk_create(arr, len(problems), ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(h)),
               "kzk_create")
        self.h = h
        self.n_inst = len(problems)
        self.offsets = [lib().kzk_inst_offset(self.h, i) for i in range(self.n_inst + 1)]
        if y_threads:
            self.set_y_threads(y_threads)
        if tau_threads:
            self.set_tau_threads(tau_threads)
        if tau_fft_radix:
            self.set_tau_fft_radix(tau_fft_radix)
        if graph:
            self.set_graph(True)

    def close(self):
        if getattr(self, "h", None):
            lib().kzk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- configuration
    def set_stream(self, stream=None):
        _check(lib().kzk_set_stream(self.h, ctypes.c_void_p(_stream_handle(stream))), "kzk_set_stream")

    def set_graph(self, on: bool):
        _check(lib().kzk_set_graph(self.h, 1 if on else 0), "kzk_set_graph")

    def set_y_threads(self, n: int):
        _check(lib().kzk_set_y_threads(self.h, int(n)), "kzk_set_y_threads")

    @property
    def y_threads(self) -> int:
        return lib().kzk_get_y_threads(self.h)

    def set_tau_threads(self, n: int):
        _check(lib().kzk_set_tau_threads(self.h, int(n)), "kzk_set_tau_threads")

    @property
    def tau_threads(self) -> int:
        return lib().kzk_get_tau_threads(self.h)

    def set_tau_fft_radix(self, r: int):
        _check(lib().kzk_set_tau_fft_radix(self.h, int(r)), "kzk_set_tau_fft_radix")

    @property
    def tau_fft_radix(self) -> int:
        return lib().kzk_get_tau_fft_radix(self.h)

    def tuning(self) -> dict:
        """The block sizes and the tau-transform radix schedule the plan runs with."""
        return {"y_threads": self.y_threads, "tau_threads": self.tau_threads, "tau_fft_radix": self.tau_fft_radix}


    # -- buffers
    @property
    def total(self) -> int:
        return self.offsets[-1]

    def _check_field(self, u):
        torch = _torch()
        if not (isinstance(u, torch.Tensor) and u.is_cuda and u.dtype == self.tdtype and u.is_contiguous()):
            raise ValueError("field must be a contiguous %s CUDA tensor" % self.tdtype)
        if u.numel() != self.total:
            raise ValueError("field has %d elements, plan needs %d" % (u.numel(), self.total))

    def pack(self, fields: Sequence[np.ndarray]):
        torch = _torch()
        flat = np.concatenate([np.ascontiguousarray(f, dtype=np.float64).ravel() for f in fields])
        return torch.from_numpy(flat).to(device="cuda", dtype=self.tdtype)

    def unpack(self, u) -> List[np.ndarray]:
        a = u.detach().double().cpu().numpy()
        out = []
        for i, p in enumerate(self.problems):
            out.append(a[self.offsets[i]:self.offsets[i + 1]].reshape(p.n_y, p.n_tau))
        return out

    # -- the method
    def step(self, u, first: int = 0, n_steps: int = 1):
        self._check_field(u)
        _check(lib().kzk_step(self.h, ctypes.c_void_p(u.data_ptr()), int(first), int(n_steps)), "kzk_step")
        return u

    def adjoint(self, u0, lam, first: int = 0, n_steps: int = 1, ckpt: int = 50, out=None):
        self._check_field(u0)
        self._check_field(lam)
        torch = _torch()
        g = torch.empty_like(lam) if out is None else out
        _check(lib().kzk_adjoint(self.h, ctypes.c_void_p(u0.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                 int(first), int(n_steps), int(ckpt), ctypes.c_void_p(g.data_ptr())),
               "kzk_adjoint")
        return g

    def profile(self, on: bool, every: int = 1):
        """Per-kernel HIP-event timing of later launches (forward steps: every
        `every`-th step); off with on=False."""
        _check(lib().kzk_profile_enable(self.h, int(every) if on else 0), "kzk_profile_enable")

    def profile_read(self):
        """{kind: (total ms, launches)} since the last read (synchronises)."""
        n = len(KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int32 * n)()
        _check(lib().kzk_profile_read(self.h, ms, cnt, n), "kzk_profile_read")
        return {KINDS[i]: (ms[i], cnt[i]) for i in range(n) if cnt[i]}

    def autotune(self, u, n_trial: int = 3) -> int:
        """Pick the fastest y-pass block size on this plan (u is only read)."""
        self._check_field(u)
        r = lib().kzk_autotune(self.h, ctypes.c_void_p(u.data_ptr()), int(n_trial))
        if r < 0:
            raise KZKError(-r, "kzk_autotune")
        return r

    def read_tables(self, inst: int = 0):
        """(E/n_y, h Phi1/n_y, h Phi2/n_y) as complex numpy arrays [n_tau/2, n_y/2+1]."""
        torch = _torch()
        p = self.problems[inst]
        M, Nh = p.n_tau // 2, p.n_y // 2 + 1
        buf = torch.empty(3 * M * Nh * 2, dtype=self.tdtype, device="cuda")
        _check(lib().kzk_read_tables(self.h, int(inst), ctypes.c_void_p(buf.data_ptr())), "kzk_read_tables")
        a = buf.double().cpu().numpy().reshape(3, M, Nh, 2)
        c = a[..., 0] + 1j * a[..., 1]
        return c[0], c[1], c[2]

    def poll(self) -> int:
        """Synchronise; return the device status code (0 = ok)."""
        return lib().kzk_poll(self.h)

    def eval_b(self, u, node: int = 0):
        self._check_field(u)
        torch = _torch()
        b = torch.empty_like(u)
        _check(lib().kzk_eval_b(self.h, ctypes.c_void_p(u.data_ptr()), int(node), ctypes.c_void_p(b.data_ptr())),
               "kzk_eval_b")
        return b

    def tau_forward(self, u):
        self._check_field(u)
        torch = _torch()
        spec = torch.empty(self.total, dtype=self.tdtype, device=u.device)   # M*n_y complex = n_tau*n_y reals
        _check(lib().kzk_tau_forward(self.h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(spec.data_ptr())),
               "kzk_tau_forward")
        return spec

    def tau_inverse(self, spec):
        torch = _torch()
        u = torch.empty(self.total, dtype=self.tdtype, device=spec.device)
        _check(lib().kzk_tau_inverse(self.h, ctypes.c_void_p(spec.data_ptr()), ctypes.c_void_p(u.data_ptr())),
               "kzk_tau_inverse")
        return u
