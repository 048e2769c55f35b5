"""Pins of the oracle on the paper's grid shape N_theta = 7 2^k (Table 0): the
mixed-radix transform against the definition of the DFT (direct sum) and
numpy, the linear part exact on such a grid (closed form), WENO5 fifth order
and ExpRK22 second order with n_tau = 7 2^k."""
import math

import numpy as np
import pytest

from paper_2103_06080_amd import inputs as I
from test_oracle_pins import rel_l2, small_problem


@pytest.mark.parametrize("n", [7, 14, 28, 56, 112])
@pytest.mark.parametrize("sign", [-1, 1])
def test_mixed_radix_fft_matches_direct_dft(orc, n, sign):
    x = I.random_field(80 + n, (n,)) + 1j * I.random_field(81 + n, (n,))
    j = np.arange(n)
    ref = (x[None, :] * np.exp(sign * 2j * np.pi * np.outer(j, j) / n)).sum(axis=1)
    got = orc.fft(x, sign)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("n", [448, 896, 1792, 3584])
def test_mixed_radix_fft_matches_numpy(orc, n):
    x = I.random_field(90, (n,)) + 1j * I.random_field(91, (n,))
    assert np.abs(orc.fft(x) - np.fft.fft(x)).max() < 1e-13 * np.abs(np.fft.fft(x)).max()


def test_linear_part_exact_on_a_7_2k_grid(orc):
    D, s, h, ns = 0.05, 1.0, 0.05, 20
    p = small_problem(nt=448, ny=64, h=h, n_steps=ns, D=D, nl=0.0)
    tau, y = p.tau(), p.y()
    k = 2 * math.pi * 5 / p.L_tau
    p.u0 = np.cos(k * tau)[None, :] * np.exp(-y ** 2 / (2 * s * s))[:, None]
    u = orc.run(p)
    c = s * s - 1j * D * h * ns / k
    ref = np.real(np.exp(1j * k * tau)[None, :] * (s / np.sqrt(c)) * np.exp(-y ** 2 / (2 * c))[:, None])
    assert rel_l2(u, ref) < 1e-12


def test_weno5_fifth_order_on_7_2k_lines(orc):
    errs = []
    for n in (112, 224, 448, 896):
        L = 8.0
        tau = -4 + L / n * np.arange(n)
        u = 0.5 + 0.25 * np.sin(2 * math.pi * tau / L)
        du = 0.25 * 2 * math.pi / L * np.cos(2 * math.pi * tau / L)
        b = orc.weno_b(u, L / n, 1.0, np.abs(u).max())
        errs.append(np.abs(b + u * du).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert min(orders[1:]) > 4.7, orders


def test_exprk22_second_order_on_a_7_2k_grid(orc):
    sols = []
    for ns in (20, 40, 80):
        p = small_problem(nt=224, ny=32, h=0.4 / ns, n_steps=ns)
        tau, y = p.tau(), p.y()
        p.u0 = (-(tau / 1.0) * 0.5 * (np.tanh((tau + 1) / 0.4) - np.tanh((tau - 1) / 0.4)))[None, :] * \
            (1 + 0.1 * np.cos(2 * np.pi * y / 16))[:, None]
        sols.append(orc.run(p))
    p_obs = math.log2(np.linalg.norm(sols[0] - sols[1]) / np.linalg.norm(sols[1] - sols[2]))
    assert 1.9 <= p_obs <= 2.6, p_obs


@pytest.mark.parametrize("m", [1, 3, 5, 9, 15])
@pytest.mark.parametrize("a", [0, 1, 3, 5])
def test_mixed_radix_fft_other_odd_factors_match_numpy(orc, m, a):
    """Lengths 2^a m for odd m other than 7: the radix-2 steps down to the
    odd factor and its direct sum, in both directions."""
    n = m << a
    x = I.random_field(100 + n, (n,)) + 1j * I.random_field(101 + n, (n,))
    ref = np.fft.fft(x)
    assert np.abs(orc.fft(x) - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())
    back = orc.fft(orc.fft(x), 1) / n
    assert np.abs(back - x).max() < 1e-13 * np.abs(x).max()


def test_adjoint_on_a_7_2k_grid_matches_central_differences(orc):
    """The oracle's discrete adjoint with mixed-radix transforms: <grad, d>
    against a central difference of L(u0) = <u(x_end), lam> along d."""
    import dataclasses
    from test_gpu_adjoint import nwave_problem
    p = nwave_problem(448, 32, 5, scheduled=True)
    lam = I.random_field(77, (32, 448))
    g = orc.adjoint(p, lam, ckpt=2)
    d = I.random_field(5, (32, 448))
    e = 1e-6

    def L(u):
        return float((orc.run(dataclasses.replace(p, u0=u)) * lam).sum())
    fd = (L(p.u0 + e * d) - L(p.u0 - e * d)) / (2 * e)
    assert abs(fd - float((g * d).sum())) < 1e-4 * abs(fd)
