"""Pins of the oracle's transport terms (the full inhomogeneous b).

b = 2 pi U_par d_tau u - U_perp d_y u + (B/2) d_tau u^2 in the paper's form
(Sec. 3.3, b of eq. (16)); in the conservative form of Sec. 3.4 eq. (21)-(22)
it is -d_tau(nl u^2/2 - 2 pi U_par u) - d_y(U_perp u) + (d_y U_perp) u, with a
WENO5/LF flux difference along each direction.  The random velocity field is
the one of Sec. 2 (Algorithm 1).  Checked against: finite differences and
the divergence-free construction of the field, the paper's bound on its
size, the energy its spectrum integrates to (closed form), a Cartesian
evaluation of the mode sum, the Burgers b where the field
vanishes, fifth-order convergence of b to its exact value on smooth data,
exact telescoping of the flux differences, exact translation by a constant
U_par, and second-order convergence of the march.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_2103_06080_amd import inputs as I
from test_oracle_pins import rel_l2, small_problem


def medium_problem(nt=64, ny=64, h=1e-3, n_steps=4, seed=7, n_modes=200, **kw):
    p = small_problem(nt=nt, ny=ny, h=h, n_steps=n_steps, **kw)
    return dataclasses.replace(p, **I.medium(seed, n_modes))


def profile_problem(nt, ny, upar, uperp, duperp, **kw):
    """x-independent velocity profiles given at the grid rows (test configuration)."""
    p = small_problem(nt=nt, ny=ny, **kw)
    return dataclasses.replace(p, vel=2, vel_prof=np.stack([upar, uperp, duperp]).astype(np.float64))


# --------------------------------------------------------------------------- the velocity field

def _sample_points(n, seed):
    u = I.splitmix_uniform_array(seed, 2 * n).reshape(n, 2)
    return 120.0 * u[:, 0], 400.0 * u[:, 1]          # the paper's (sigma, rho) domain


def test_velocity_field_is_divergence_free(orc):
    """U~_n . K_n = 0 makes U = sum U~_n cos(K_n . r + phi_n) divergence free:
    d_x U_par + d_y U_perp = 0 (central differences, step e)."""
    p = medium_problem()
    e = 1e-4
    for x, y in zip(*_sample_points(20, 3)):
        ddx = (orc.velocity(p, x + e, y)[0] - orc.velocity(p, x - e, y)[0]) / (2 * e)
        ddy = (orc.velocity(p, x, y + e)[1] - orc.velocity(p, x, y - e)[1]) / (2 * e)
        assert abs(ddx + ddy) < 1e-7 * max(1.0, abs(ddx)) + 1e-9, (x, y, ddx, ddy)
        assert abs(ddx) > 1e-6          # the field does vary


def test_velocity_derivative_matches_finite_difference(orc):
    p = medium_problem()
    e = 1e-4
    for x, y in zip(*_sample_points(20, 4)):
        fd = (orc.velocity(p, x, y + e)[1] - orc.velocity(p, x, y - e)[1]) / (2 * e)
        assert abs(orc.velocity(p, x, y)[2] - fd) < 1e-8 * max(1.0, abs(fd)) + 1e-10


def test_velocity_field_is_bounded_as_stated(orc):
    """The paper's parameters give ||U_par||, ||U_perp|| <= 0.05 (Sec. 2)."""
    p = medium_problem(n_modes=200)
    xs = np.linspace(0, 120, 61)
    ys = np.linspace(0, 400, 201)
    v = np.array([[orc.velocity(p, x, y)[:2] for y in ys] for x in xs])
    assert np.abs(v).max() <= 0.05
    assert np.abs(v).max() > 0.01
    assert abs(v[..., 0].mean()) < 0.01 and abs(v[..., 1].mean()) < 0.01


def test_velocity_equals_cartesian_mode_sum(orc):
    """The polar form of Algorithm 1 equals sum_n U~_n cos(K_n . r + phi_n) with
    K_n . r = K_n lambda (x cos theta_n + y sin theta_n)."""
    p = medium_problem(n_modes=50)
    L = 4 * p.vel_lambda
    K = np.linspace(0.1 / L, 9.0 / L, p.vel_modes)
    E = p.vel_sigma_u ** 2 * K ** 3 * L ** 4 * np.exp(-(K * L / 2) ** 2) / 8
    amp = np.sqrt(E / p.vel_modes) / p.vel_c0
    for x, y in zip(*_sample_points(10, 5)):
        ph = K * p.vel_lambda * (x * np.cos(p.vel_theta) + y * np.sin(p.vel_theta)) + p.vel_phi
        ref = [np.sum(-amp * np.sin(p.vel_theta) * np.cos(ph)), np.sum(amp * np.cos(p.vel_theta) * np.cos(ph))]
        got = orc.velocity(p, x, y)
        assert abs(got[0] - ref[0]) < 1e-12 and abs(got[1] - ref[1]) < 1e-12


# --------------------------------------------------------------------------- b with transport

def test_transport_b_without_velocity_is_the_burgers_b(orc):
    nt, ny = 128, 16
    z = np.zeros(ny)
    p = profile_problem(nt, ny, z, z, z, nl=0.8)
    u = I.random_field(61, (ny, nt))
    b = orc.eval_b(p, 0.0, 0.8, u)
    ref = np.stack([orc.weno_b(u[j], p.dtau, 0.8, 0.8 * np.abs(u[j]).max()) for j in range(ny)])
    assert np.abs(b - ref).max() == 0.0


def _smooth_case(n):
    Lt, Ly = 8.0, 16.0
    p0 = small_problem(nt=n, ny=n, Lt=Lt, Ly=Ly, nl=0.7)
    tau, y = p0.tau(), p0.y()
    ky = 2 * np.pi / Ly
    upar = 0.03 * np.cos(ky * (y - p0.y0))
    uperp = 0.04 * np.sin(ky * (y - p0.y0) + 0.3)
    duperp = 0.04 * ky * np.cos(ky * (y - p0.y0) + 0.3)
    p = profile_problem(n, n, upar, uperp, duperp, nl=0.7, Lt=Lt, Ly=Ly)
    a, c = 2 * np.pi / Lt, ky
    T, Y = np.meshgrid(tau, y - p0.y0)
    u = 0.5 + 0.25 * np.sin(a * T) * np.cos(c * Y)
    u_t = 0.25 * a * np.cos(a * T) * np.cos(c * Y)
    u_y = -0.25 * c * np.sin(a * T) * np.sin(c * Y)
    exact = -0.7 * u * u_t + 2 * np.pi * upar[:, None] * u_t - uperp[:, None] * u_y
    return p, u, exact


def test_transport_b_converges_at_fifth_order(orc):
    errs = []
    ns = [32, 64, 128]
    for n in ns:
        p, u, exact = _smooth_case(n)
        b = orc.eval_b(p, 0.0, 0.7, u)
        errs.append(np.abs(b - exact).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 4.5, orders


def test_transport_flux_differences_telescope(orc):
    """Sum over the field of b = sum of the source (d_y U_perp) u: the tau and y
    flux differences of a periodic field sum to zero."""
    p = medium_problem(nt=128, ny=64)
    u = I.random_field(62, (64, 128)) + 0.2
    x = 0.37
    b = orc.eval_b(p, x, 0.9, u)
    src = np.array([orc.velocity(p, x, yj)[2] for yj in p.y()])[:, None] * u
    assert abs(b.sum() - src.sum()) < 1e-10 * np.abs(b).sum()


def test_constant_axial_velocity_translates_in_tau(orc):
    """nl = 0, D = 0, A = 0, U_perp = 0, U_par = c: u_x = 2 pi c u_tau, so
    u(x, tau) = u0(tau + 2 pi c x) (WENO5 in tau, ExpRK22 in x)."""
    nt, ny, cpar = 256, 8, 0.04
    one = np.ones(ny)
    p = profile_problem(nt, ny, cpar * one, 0 * one, 0 * one, nl=0.0, D=0.0, h=2e-3, n_steps=100)
    tau = p.tau()
    p.u0 = np.tile(np.exp(-4 * np.sin(np.pi * (tau - p.tau0) / p.L_tau) ** 2), (ny, 1))
    u = orc.run(p)
    X = p.h * p.n_steps
    ref = np.tile(np.exp(-4 * np.sin(np.pi * (tau + 2 * np.pi * cpar * X - p.tau0) / p.L_tau) ** 2), (ny, 1))
    assert rel_l2(u, ref) < 1e-5


def test_march_with_transport_is_second_order(orc):
    sols = []
    X = 0.4
    for ns in (20, 40, 80):
        p = medium_problem(nt=128, ny=64, h=X / ns, n_steps=ns, n_modes=30)
        tau, y = p.tau(), p.y()
        p.u0 = (-(tau / 1.0) * 0.5 * (np.tanh((tau + 1) / 0.4) - np.tanh((tau - 1) / 0.4)))[None, :] * \
            (1 + 0.1 * np.cos(2 * np.pi * y / 16))[:, None]
        sols.append(orc.run(p))
    p_obs = math.log2(np.linalg.norm(sols[0] - sols[1]) / np.linalg.norm(sols[1] - sols[2]))
    assert 1.85 <= p_obs <= 2.6, p_obs


# --------------------------------------------------------------------------- exact rational checks

def _exact_lf_line(f, a, dx, eps):
    """-(F_{i+1/2} - F_{i-1/2}) / dx on a periodic line of flux values f and
    speed a, F = F+ + F- from the WENO5 definitions in exact arithmetic."""
    from fractions import Fraction as Fr
    import test_oracle_weno_exact as X
    n = len(f)
    a, dx, eps = Fr(a), Fr(dx), Fr(eps)
    fp = [(fj + a * uj) / 2 for fj, uj in f]
    fm = [(fj - a * uj) / 2 for fj, uj in f]
    F = []
    for i in range(n):
        F.append(X.face_value([fp[(i - 2 + r) % n] for r in range(5)], eps)[0] +
                 X.face_value([fm[(i + 3 - r) % n] for r in range(5)], eps)[0])
    return [-(F[i] - F[i - 1]) / dx for i in range(n)]


def test_axial_transport_term_equals_exact_evaluation(orc):
    """Rough field, U_perp = 0, U_par varying from row to row: each tau-line's
    flux is nl u^2/2 - 2 pi U_par u with the LF speed max |nl u - 2 pi U_par|."""
    from fractions import Fraction as Fr
    nt, ny, nl = 16, 3, 0.8
    upar = np.array([0.04, -0.03, 0.0])
    p = profile_problem(nt, ny, upar, np.zeros(ny), np.zeros(ny), nl=nl)
    u = np.where(np.arange(nt) % 5 < 2, 1.0, -0.3)[None, :] + 0.1 * I.random_field(71, (ny, nt))
    b = orc.eval_b(p, 0.0, nl, u)
    for j in range(ny):
        c = 2 * np.pi * upar[j]
        U = [Fr(float(x)) for x in u[j]]
        C = Fr(float(c))
        f = [(Fr(nl) * x * x / 2 - C * x, x) for x in U]
        a = max(abs(Fr(nl) * x - C) for x in U)
        ref = np.array([float(v) for v in _exact_lf_line(f, a, p.dtau, p.weno_eps)])
        assert np.abs(b[j] - ref).max() <= 1e-13 * np.abs(ref).max(), j


def test_transverse_transport_term_equals_exact_evaluation(orc):
    """Rough field, nl = 0, U_par = 0, U_perp and d_y U_perp arbitrary per row:
    b = -(G_{j+1/2} - G_{j-1/2}) / dy + (d_y U_perp)_j u_j along every y-line,
    G from g = U_perp u with the LF speed max_j |U_perp(y_j)|."""
    from fractions import Fraction as Fr
    nt, ny = 4, 14
    uperp = 0.05 * I.random_field(72, (ny,))
    duperp = 0.3 * I.random_field(73, (ny,))
    p = profile_problem(nt, ny, np.zeros(ny), uperp, duperp, nl=0.0)
    u = np.where(np.arange(ny) % 6 < 2, 0.9, -0.5)[:, None] + 0.1 * I.random_field(74, (ny, nt))
    b = orc.eval_b(p, 0.0, 0.0, u)
    dy = p.L_y / ny
    a = max(abs(Fr(float(v))) for v in uperp)
    for k in range(nt):
        U = [Fr(float(x)) for x in u[:, k]]
        f = [(Fr(float(uperp[j])) * U[j], U[j]) for j in range(ny)]
        ref = _exact_lf_line(f, a, dy, p.weno_eps)
        ref = np.array([float(ref[j] + Fr(float(duperp[j])) * U[j]) for j in range(ny)])
        assert np.abs(b[:, k] - ref).max() <= 1e-13 * np.abs(ref).max(), k


def test_velocity_field_carries_the_energy_of_its_spectrum(orc):
    """The spectrum E(K) = sigma_u^2 K^3 L^4 exp(-(K L / 2)^2) / 8 integrates to
    sigma_u^2 over K >= 0 (closed form: int K^3 e^{-a K^2} dK = 1/(2 a^2),
    a = L^2/4).  With N modes equispaced in [0.1/L, 9/L] (spacing dK) and
    |U~_n|^2 = E(K_n) / N / c0^2, the field's mean square over the plane is
    sum_n |U~_n|^2 / 2 = (sum_n E(K_n) dK) / (2 N dK c0^2), i.e. sigma_u^2 /
    (2 N dK c0^2) up to the Riemann sum; checked on a spatial average over a
    large window (sampling error a few per cent), which catches a wrong
    amplitude normalisation (a missing square root, 1/N or 1/2)."""
    p = medium_problem(n_modes=200, seed=11)
    L = 4 * p.vel_lambda
    dK = (9.0 / L - 0.1 / L) / (p.vel_modes - 1)
    want = p.vel_sigma_u ** 2 / (2 * p.vel_modes * dK * p.vel_c0 ** 2)
    u = I.splitmix_uniform_array(21, 2 * 4000).reshape(4000, 2)
    xs, ys = 5000.0 * u[:, 0], 5000.0 * u[:, 1]
    v = np.array([orc.velocity(p, x, y)[:2] for x, y in zip(xs, ys)])
    got = float((v ** 2).sum(axis=1).mean())
    assert abs(got / want - 1) < 0.1, (got, want)
