"""Pins of the oracle's two method variants (Sec. 3.3 and Sec. 3.4):

* exponential Euler, the first-order member of the family
  (u^{n+1} = E u^n + h phi1(hL) b(x_n, u^n)): exact for a forcing that does
  not depend on u or x, first order in h otherwise;
* the regularised Fourier multiplier of the definition of z_jk, where the
  antiderivative 1/(i k_tau) becomes 1/(i k_tau + eps/(4 pi)), so that the
  mean tau-mode takes the same formula as every other mode (instead of
  being zeroed) and F(b) keeps its mean mode.

Each is checked against something other than the oracle: closed forms of the
linear problem per Fourier mode (numpy FFTs, scipy expm of the augmented
system), the unregularised method where the two must agree, and observed
convergence orders.
"""
import dataclasses
import math

import numpy as np
import scipy.linalg

from paper_2103_06080_amd import inputs as I
from test_oracle_pins import I_avg, nw_smooth, rel_l2, small_problem

EPS64, EPS32 = 2.0 ** -53, 2.0 ** -24


def variant(p, **kw):
    return dataclasses.replace(p, **kw)


# --------------------------------------------------------------------------- exponential Euler

def test_exponential_euler_exact_for_constant_forcing(orc):
    """b = beta0 (u- and x-independent): u(x) = e^{xL} u0 + x phi1(xL) beta0
    exactly, for any h; reference per Fourier mode from the matrix
    exponential of d/dx [u, 1] = [[l, B0], [0, 0]] [u, 1]."""
    nt, ny, h, ns = 32, 16, 0.07, 6
    p = variant(small_problem(nt=nt, ny=ny, h=h, n_steps=ns, D=0.09, nl=0.0, A=3e-3), scheme=1)
    p.u0 = I.random_field(21, (ny, nt))
    f0 = I.random_field(22, (ny, nt))
    f0 -= f0.mean(axis=1, keepdims=True)      # F(b)(0, .) is zeroed by the unregularised multiplier
    u = orc.run(p, force0=f0, force1=np.zeros_like(f0))
    U0, B0 = np.fft.fft2(p.u0), np.fft.fft2(f0)
    kt = 2 * np.pi * np.fft.fftfreq(nt, d=p.L_tau / nt)
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=p.L_y / ny)
    X = h * ns
    out = np.zeros_like(U0)
    for n in range(ny):
        for m in range(nt):
            l = 0.0 if m == 0 else (-p.A * kt[m] ** 2 if 2 * m == nt
                                    else 1j * 0.09 * ky[n] ** 2 / (2 * kt[m]) - p.A * kt[m] ** 2)
            Mx = np.array([[l, B0[n, m]], [0, 0]], dtype=complex)
            out[n, m] = (scipy.linalg.expm(Mx * X) @ np.array([U0[n, m], 1.0]))[0]
    ref = np.real(np.fft.ifft2(out))
    assert rel_l2(u, ref) < 1e-12


def test_exponential_euler_not_exact_for_x_dependent_forcing(orc):
    """With b = beta0 + x beta1 the first-order method leaves an O(h) error
    (ExpRK22, second order, integrates this forcing exactly)."""
    nt, ny = 32, 16
    errs = []
    for ns in (8, 16):
        p = small_problem(nt=nt, ny=ny, h=0.4 / ns, n_steps=ns, D=0.05, nl=0.0, A=1e-3)
        p.u0 = I.random_field(31, (ny, nt))
        f0 = I.random_field(32, (ny, nt))
        f1 = I.random_field(33, (ny, nt))
        f0 -= f0.mean(axis=1, keepdims=True)
        f1 -= f1.mean(axis=1, keepdims=True)
        exact = orc.run(p, force0=f0, force1=f1)             # ExpRK22: exact for this forcing
        ee = orc.run(variant(p, scheme=1), force0=f0, force1=f1)
        errs.append(np.linalg.norm(ee - exact))
    ratio = errs[0] / errs[1]
    assert 1.8 < ratio < 2.2, ratio


def test_exponential_euler_first_order(orc):
    sols = []
    X = 0.4
    for ns in (20, 40, 80):
        h = X / ns
        xn = h * np.arange(ns + 1)
        p = variant(small_problem(nt=128, ny=64, h=h, n_steps=ns), scheme=1)
        p.D_step = np.array([I_avg(lambda x: 0.05 + 0 * x, x, h) for x in xn[:-1]])
        p.nl_node = np.ones(ns + 1)
        p.u0 = nw_smooth(p.tau(), p.y())
        sols.append(orc.run(p))
    p_obs = math.log2(np.linalg.norm(sols[0] - sols[1]) / np.linalg.norm(sols[1] - sols[2]))
    assert 0.9 <= p_obs <= 1.15, p_obs


# --------------------------------------------------------------------------- regularised multiplier

def test_regularised_equals_unregularised_on_fields_of_zero_tau_mean(orc):
    """Away from k_tau = 0 the shift eps/(4 pi) changes the symbol by a relative
    O(eps/k_tau); on fields whose rows have zero tau-mean (b has none either)
    the two multipliers give the same march."""
    p = small_problem(nt=128, ny=64, h=2e-3, n_steps=30, D=0.05, nl=1.0, A=1e-3)
    p.u0 = nw_smooth(p.tau(), p.y())
    p.u0 -= p.u0.mean(axis=1, keepdims=True)
    a = orc.run(p)
    for eps in (EPS64, EPS32):
        b = orc.run(variant(p, reg_eps=eps))
        assert rel_l2(b, a) < 1e-13, eps


def test_regularised_multiplier_removes_the_y_varying_tau_mean(orc):
    """At k_tau = 0, ky != 0 the regularised symbol is -(D/2) ky^2 (4 pi / eps),
    so with eps = 2^-53 one step multiplies those modes by e^{z}, which is 0 in
    FP64: afterwards every row has the same tau-mean, the y-average of the
    initial ones.  The unregularised multiplier (l = 0 there) keeps each row's
    mean."""
    nt, ny = 64, 32
    p = small_problem(nt=nt, ny=ny, h=1e-3, n_steps=3, D=0.05, nl=0.0, A=0.0)
    y = p.y()
    g = 0.4 + 0.3 * np.cos(2 * np.pi * (y - p.y0) / p.L_y) + 0.2 * np.sin(6 * np.pi * (y - p.y0) / p.L_y)
    zm = I.random_field(41, (ny, nt))
    zm -= zm.mean(axis=1, keepdims=True)
    p.u0 = g[:, None] + zm
    kept = orc.run(p)
    assert np.abs(kept.mean(axis=1) - g).max() < 1e-14
    reg = orc.run(variant(p, reg_eps=EPS64))
    assert np.abs(reg.mean(axis=1) - g.mean()).max() < 1e-14
    # the rest of the field evolves as before
    assert rel_l2(reg - reg.mean(axis=1, keepdims=True), kept - kept.mean(axis=1, keepdims=True)) < 1e-13


def test_regularised_mean_column_follows_its_closed_form(orc):
    """With eps = 2^-24 and a small step the mean-mode multipliers are neither
    0 nor 1: the tau-mean column, transformed along y, decays mode by mode as
    exp(x l_0(n)), l_0(n) = -(D/2) ky^2 (4 pi / eps) (linear problem, exact
    for any h)."""
    nt, ny, h, ns, D = 32, 32, 4e-7, 5, 0.02
    p = variant(small_problem(nt=nt, ny=ny, h=h, n_steps=ns, D=D, nl=0.0, A=0.0), reg_eps=EPS32)
    y = p.y()
    g = sum(0.1 * (k + 1) * np.cos(2 * np.pi * k * (y - p.y0) / p.L_y + 0.3 * k) for k in range(5))
    p.u0 = g[:, None] + 0.0 * p.tau()[None, :]
    u = orc.run(p)
    got = np.fft.fft(u.mean(axis=1))
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=p.L_y / ny)
    l0 = -(D / 2) * ky ** 2 * (4 * np.pi / EPS32)
    ref = np.exp(h * ns * l0) * np.fft.fft(g)
    decay = np.exp(h * ns * l0[1:4])
    assert decay.min() > 1e-4 and decay.max() < 0.9      # the step resolves the decay
    assert np.abs(got - ref).max() < 1e-13 * np.abs(np.fft.fft(g)).max()


def test_regularised_multiplier_keeps_the_mean_of_b(orc):
    """The regularised multiplier keeps F(b)(0, 0): a forcing with a global
    mean m raises the mean of u by x m (l = 0 and phi1 = 1 there); the
    unregularised one zeroes it and the mean stays."""
    nt, ny, h, ns = 32, 16, 0.01, 7
    p = small_problem(nt=nt, ny=ny, h=h, n_steps=ns, D=0.05, nl=0.0, A=1e-3)
    p.u0 = I.random_field(51, (ny, nt))
    f0 = I.random_field(52, (ny, nt)) * 0.1 + 0.25
    zero = np.zeros_like(f0)
    kept = orc.run(p, force0=f0, force1=zero)
    reg = orc.run(variant(p, reg_eps=EPS64), force0=f0, force1=zero)
    assert abs(kept.mean() - p.u0.mean()) < 1e-15
    assert abs(reg.mean() - (p.u0.mean() + h * ns * f0.mean())) < 1e-14
