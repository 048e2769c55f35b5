"""Seeded synthetic inputs for the KZK exponential-integrator/WENO5 step.

This module holds no arithmetic of the method itself: it only draws numbers
and builds the initial fields and coefficient schedules that both the HIP
path and the CPU oracle take as inputs.

Workloads (the paper runs an N-wave pulse, Sec. 4, through a random medium
whose realisation is not published; these synthetic N-waves stand in for it):

* ``c1``  plain method, 256 x 128, D = 0.05, h = 1e-3, 200 steps, seed-free;
* ``c2``  homogeneous medium, 4096 x 2048, D = 0.02, h = 5e-4, 1000 steps;
* ``c3``  inhomogeneous coefficients nl(x) = 1 + 0.5 tanh(x - 2),
          D(x) = 0.02 (1 + 0.3 sin x), A = 1e-4, 8192 x 4096, h = 2.5e-4, 2000 steps;
* ``c4``  64 independent solves of uneven size, tau in {512, 1024, 2048},
          y in {256, 512, 1024}, D ~ U[0.01, 0.05], h = 5e-4, 500 steps;
* ``c5``  adjoint workload, 2048 x 1024, D = 0.03, h = 5e-4, 500 steps, K = 50.

Random numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014):
state += 0x9E3779B97F4A7C15, then the two xor-shift-multiply mixing rounds;
a uniform double is (x >> 11) * 2^-53.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def _mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


class SplitMix64:
    """Sequential SplitMix64 stream (scalar draws in a documented order)."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + _GAMMA) & _MASK
        return _mix(self.state)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * 2.0 ** -53

    def uniform_range(self, lo: float, hi: float) -> float:
        return lo + (hi - lo) * self.uniform()

    def integer(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi]."""
        return lo + min(int(self.uniform() * (hi - lo + 1)), hi - lo)


def splitmix_uniform_array(seed: int, n: int) -> np.ndarray:
    """The first n uniforms of SplitMix64(seed), vectorised (same values as the
    scalar stream: output i mixes seed + (i+1) * gamma)."""
    with np.errstate(over="ignore"):
        i = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed & _MASK) + i * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def splitmix_normal_array(seed: int, n: int) -> np.ndarray:
    """n standard normals by the Box-Muller transform of SplitMix64 uniforms."""
    m = (n + 1) // 2
    u = splitmix_uniform_array(seed, 2 * m)
    u1 = 1.0 - u[0::2]                 # (0, 1]
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.concatenate([r * np.cos(2 * math.pi * u2), r * np.sin(2 * math.pi * u2)])
    return z[:n]


@dataclasses.dataclass
class Problem:
    """One solve: grid, coefficients and initial field (u0[y, tau], tau contiguous)."""

    name: str
    n_tau: int
    n_y: int
    h: float
    n_steps: int
    D_step: np.ndarray          # [n_steps]   diffraction coefficient used in step n
    nl_node: np.ndarray         # [n_steps+1] Burgers coefficient at x_n
    u0: np.ndarray              # [n_y, n_tau] float64
    tau0: float = -4.0
    L_tau: float = 8.0
    y0: float = -8.0
    L_y: float = 16.0
    x0: float = 0.0
    A: float = 0.0
    weno_eps: float = 1e-6
    lf_scope: int = 0           # 0: LF speed per tau-line, 1: global
    D_const: Optional[float] = None
    nl_const: Optional[float] = None
    scheme: int = 0             # 0: ExpRK22; 1: exponential Euler
    reg_eps: float = 0.0        # 0: mean tau-mode zeroed; > 0: regularised multiplier with this epsilon
    # transport by a velocity field: vel = 0 none, 1 the random field of Sec. 2
    # (vel_modes modes with phases vel_phi and angles vel_theta), 2 fixed
    # profiles vel_prof[3][n_y] (U_par, U_perp, d_y U_perp; oracle tests only)
    vel: int = 0
    vel_modes: int = 0
    vel_phi: Optional[np.ndarray] = None
    vel_theta: Optional[np.ndarray] = None
    vel_lambda: float = 6.86    # lambda = T0 c0 (m): T0 = 0.02 s, c0 = 343 m/s
    vel_sigma_u: float = 3.0    # sigma_u (m/s)
    vel_c0: float = 343.0       # ambient sound speed (m/s), U is normalised by it
    vel_prof: Optional[np.ndarray] = None

    @property
    def dtau(self) -> float:
        return self.L_tau / self.n_tau

    @property
    def points(self) -> int:
        return self.n_tau * self.n_y

    def tau(self) -> np.ndarray:
        return self.tau0 + self.dtau * np.arange(self.n_tau)

    def y(self) -> np.ndarray:
        return self.y0 + (self.L_y / self.n_y) * np.arange(self.n_y)

    def with_steps(self, n_steps: int) -> "Problem":
        """Same problem truncated (or extended, for constant coefficients) to n_steps."""
        if n_steps <= self.n_steps:
            return dataclasses.replace(self, n_steps=n_steps, D_step=self.D_step[:n_steps].copy(),
                                       nl_node=self.nl_node[:n_steps + 1].copy())
        if self.D_const is None or self.nl_const is None:
            raise ValueError("cannot extend a problem with x-dependent coefficients")
        return dataclasses.replace(self, n_steps=n_steps, D_step=np.full(n_steps, self.D_const),
                                   nl_node=np.full(n_steps + 1, self.nl_const))


def nwave(tau: np.ndarray, y: np.ndarray, T: float, a: float, w: float,
          modes: List[tuple], y0: float, L_y: float) -> np.ndarray:
    """Smoothed N-wave -a (tau/T) on |tau| < T with tanh edges of width w, times
    the transverse modulation m(y) = 1 + sum_i a_i cos(2 pi n_i (y - y0)/L_y + phi_i)
    (the construction of the initial pulse of Sec. 4 with its edge width w)."""
    t = tau[None, :]
    ramp = -a * (t / T) * 0.5 * (np.tanh((t + T) / w) - np.tanh((t - T) / w))
    m = np.ones_like(y)
    for (amp, n, ph) in modes:
        m = m + amp * np.cos(2 * math.pi * n * (y - y0) / L_y + ph)
    return ramp * m[:, None]


def _draw_nwave(rng: SplitMix64):
    """Draw order: T, a, then (a_i, n_i, phi_i) for the 8 cosine modes."""
    T = rng.uniform_range(0.5, 1.5)
    a = rng.uniform_range(0.5, 2.0)
    modes = []
    for _ in range(8):
        amp = rng.uniform_range(0.0, 0.05)
        n = rng.integer(1, 8)
        ph = rng.uniform_range(0.0, 2 * math.pi)
        modes.append((amp, n, ph))
    return T, a, modes


def _const_problem(name, n_tau, n_y, h, n_steps, D, nl, u0, **kw) -> Problem:
    return Problem(name=name, n_tau=n_tau, n_y=n_y, h=h, n_steps=n_steps,
                   D_step=np.full(n_steps, float(D)), nl_node=np.full(n_steps + 1, float(nl)),
                   u0=u0, D_const=float(D), nl_const=float(nl), **kw)


def c1(n_steps: int = 200) -> Problem:
    """Plain method: 256 x 128, D = 0.05, T = 1, a = 1, m(y) = 1 + 0.1 cos(2 pi y/16)."""
    p = Problem(name="c1", n_tau=256, n_y=128, h=1e-3, n_steps=0, D_step=np.zeros(0),
                nl_node=np.zeros(1), u0=np.zeros((1, 1)))
    u0 = nwave(p.tau(), p.y(), T=1.0, a=1.0, w=0.05, modes=[(0.1, 1, 0.0)], y0=0.0, L_y=16.0)
    return _const_problem("c1", 256, 128, 1e-3, n_steps, 0.05, 1.0, u0)


def _seeded(name, seed, n_tau, n_y, h, n_steps, D, **kw) -> Problem:
    rng = SplitMix64(seed)
    T, a, modes = _draw_nwave(rng)
    p = Problem(name=name, n_tau=n_tau, n_y=n_y, h=h, n_steps=0, D_step=np.zeros(0),
                nl_node=np.zeros(1), u0=np.zeros((1, 1)))
    u0 = nwave(p.tau(), p.y(), T, a, 0.05, modes, p.y0, p.L_y)
    return _const_problem(name, n_tau, n_y, h, n_steps, D, 1.0, u0, **kw)


def c2(seed: int = 0, n_steps: int = 1000, n_tau: int = 4096, n_y: int = 2048) -> Problem:
    """Homogeneous medium: 4096 x 2048, D = 0.02, h = 5e-4, 1000 steps."""
    return _seeded("c2", seed, n_tau, n_y, 5e-4, n_steps, 0.02)


def c3_coefficients(h: float, n_steps: int, x0: float = 0.0):
    """nl at the nodes x_n and the step average of D(x) = 0.02 (1 + 0.3 sin x)
    over [x_n, x_n + h]: the integral of the sine, (cos x_n - cos(x_n + h)) / h,
    written as the product 2 sin(x_n + h/2) sin(h/2) / h, which does not cancel
    for small h."""
    xn = x0 + h * np.arange(n_steps + 1)
    nl = 1.0 + 0.5 * np.tanh(xn - 2.0)
    xs = xn[:-1]
    Dbar = 0.02 * (1.0 + 0.3 * 2.0 * np.sin(xs + 0.5 * h) * np.sin(0.5 * h) / h)
    return Dbar, nl


def c3(seed: int = 0, n_steps: int = 2000, n_tau: int = 8192, n_y: int = 4096) -> Problem:
    """Inhomogeneous coefficients, absorption A = 1e-4: 8192 x 4096, h = 2.5e-4."""
    rng = SplitMix64(seed)
    T, a, modes = _draw_nwave(rng)
    h = 2.5e-4
    Dbar, nl = c3_coefficients(h, n_steps)
    p = Problem(name="c3", n_tau=n_tau, n_y=n_y, h=h, n_steps=n_steps, D_step=Dbar,
                nl_node=nl, u0=np.zeros((1, 1)), A=1e-4)
    p.u0 = nwave(p.tau(), p.y(), T, a, 0.05, modes, p.y0, p.L_y)
    return p


def c4(seed: int = 0, n_inst: int = 64, n_steps: int = 500,
       taus=(512, 1024, 2048), ys=(256, 512, 1024)) -> List[Problem]:
    """64 independent N-wave solves of uneven size; per instance, in order:
    n_tau, n_y (uniform choices), T, a, D ~ U[0.01, 0.05], 8 cosine modes."""
    rng = SplitMix64(seed)
    out = []
    for i in range(n_inst):
        nt = taus[rng.integer(0, len(taus) - 1)]
        ny = ys[rng.integer(0, len(ys) - 1)]
        T = rng.uniform_range(0.5, 1.5)
        a = rng.uniform_range(0.5, 2.0)
        D = rng.uniform_range(0.01, 0.05)
        modes = []
        for _ in range(8):
            modes.append((rng.uniform_range(0.0, 0.05), rng.integer(1, 8),
                          rng.uniform_range(0.0, 2 * math.pi)))
        p = Problem(name=f"c4[{i}]", n_tau=nt, n_y=ny, h=5e-4, n_steps=0, D_step=np.zeros(0),
                    nl_node=np.zeros(1), u0=np.zeros((1, 1)))
        u0 = nwave(p.tau(), p.y(), T, a, 0.05, modes, p.y0, p.L_y)
        out.append(_const_problem(f"c4[{i}]", nt, ny, 5e-4, n_steps, D, 1.0, u0))
    return out


def c5(seed: int = 0, n_steps: int = 500, n_tau: int = 2048, n_y: int = 1024) -> Problem:
    """Adjoint workload: 2048 x 1024, D = 0.03, h = 5e-4, 500 steps (checkpoint every 50)."""
    return _seeded("c5", seed, n_tau, n_y, 5e-4, n_steps, 0.03)


C5_CKPT = 50
C5_FD_EPS = 1e-6
C5_N_DIRECTIONS = 32
C5_KAPPA = 20.0
C5_WINDOW = (-2.0, 2.0)


def medium(seed: int, n_modes: int = 200) -> dict:
    """Random numbers of the velocity field of Sec. 2: per mode n, in order,
    the phase phi_n and the angle theta_n, both uniform in [0, 2 pi)
    (Algorithm 1 draws them as two independent sequences; here they are
    interleaved draws of one SplitMix64 stream).  Returned as Problem fields."""
    u = splitmix_uniform_array(seed, 2 * n_modes).reshape(n_modes, 2) * (2 * math.pi)
    return dict(vel=1, vel_modes=n_modes, vel_phi=u[:, 0].copy(), vel_theta=u[:, 1].copy())


# Table 0 of the paper (N_sigma, N_rho, N_theta) and the grids used for them
# here (n_tau x n_y = theta x rho): n_tau = N_theta itself (7 * 2^k), n_y the
# power of two nearest N_rho (the y-transform takes powers of two); the
# power-of-two grids nearest both are kept as a second stand-in
PAPER_SETS = {1: (300, 1250, 448), 2: (600, 2500, 896), 3: (1200, 5000, 1792), 4: (2400, 10000, 3584)}
PAPER_SET_GRIDS = {1: (448, 1024), 2: (896, 2048), 3: (1792, 4096), 4: (3584, 8192)}
PAPER_SET_POW2_GRIDS = {1: (512, 1024), 2: (1024, 2048), 3: (2048, 4096), 4: (4096, 8192)}


def paper_set(k: int, seed: int = 0, n_modes: int = 200, reg_eps: float = 2.0 ** -24,
              n_steps: Optional[int] = None, pow2: bool = False) -> Problem:
    """The paper's workload (Sec. 4) on the grid of set k of Table 0
    (PAPER_SET_GRIDS: N_theta tau-points, the power of two nearest N_rho
    rows; pow2=True: PAPER_SET_POW2_GRIDS): sigma in [0, 120] with N_sigma
    steps, rho in [0, 400),
    theta in [-13 pi, 15 pi), D/2 = 1/(4 pi), B = 0.05 (nl = -B), A = 3.4e-4,
    the random medium of Sec. 2 (seeded phases and angles), the regularised
    multiplier, and the paper's N-wave
    V0 = (theta - 3 pi)/(2 pi) (tanh(B/(4A)(theta - 4 pi)) - tanh(B/(4A)(theta - 2 pi)))."""
    n_sigma, _, _ = PAPER_SETS[k]
    n_tau, n_y = (PAPER_SET_POW2_GRIDS if pow2 else PAPER_SET_GRIDS)[k]
    ns = n_sigma if n_steps is None else n_steps
    B, A = 0.05, 3.4e-4
    p = Problem(name="paper_set%d" % k, n_tau=n_tau, n_y=n_y, h=120.0 / n_sigma, n_steps=ns,
                D_step=np.full(ns, 1.0 / (2 * math.pi)), nl_node=np.full(ns + 1, -B), u0=np.zeros((1, 1)),
                tau0=-13 * math.pi, L_tau=28 * math.pi, y0=0.0, L_y=400.0, A=A,
                D_const=1.0 / (2 * math.pi), nl_const=-B, reg_eps=reg_eps, **medium(seed, n_modes))
    th = p.tau()
    v = (th - 3 * math.pi) / (2 * math.pi) * (np.tanh(B / (4 * A) * (th - 4 * math.pi)) -
                                              np.tanh(B / (4 * A) * (th - 2 * math.pi)))
    p.u0 = np.tile(v, (n_y, 1))
    return p


def fd_direction(r: int, shape) -> np.ndarray:
    """Finite-difference direction r of the adjoint workload: N(0,1), seed 1000 + r."""
    n = int(np.prod(shape))
    return splitmix_normal_array(1000 + r, n).reshape(shape)


def random_field(seed: int, shape, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Uniform random test field (used for invariants and small parity cases)."""
    n = int(np.prod(shape))
    return (lo + (hi - lo) * splitmix_uniform_array(seed, n)).reshape(shape)


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c5": c5}
