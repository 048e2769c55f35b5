"""Pins of the oracle's WENO5 discretisation of b against its definition, in
exact rational arithmetic.

The finite-difference WENO5 scheme (Jiang and Shu 1996; Shu 1998, the WENO
reference of Sec. 3.4) treats the point values f_j of the split flux as the
cell averages of a function h and reconstructs h at the face x_{i+1/2}:

* on each candidate stencil S_r = {i-2+r, i-1+r, i+r} (r = 0, 1, 2) the
  quadratic p_r with those three cell averages gives q_r = p_r(x_{i+1/2});
* the quartic through all five cell averages gives the fifth-order value,
  which equals d_0 q_0 + d_1 q_1 + d_2 q_2 for the ideal weights d_r;
* the smoothness indicator is
  beta_r = sum_{l=1,2} dx^(2l-1) int over cell i of (d^l p_r / dx^l)^2 dx;
* the nonlinear weights are a_r = d_r / (eps + beta_r)^2, normalised.

Everything below is built from these definitions with Fractions (polynomials
solved from their cell averages and integrated exactly), never from the
closed forms of q_r and beta_r that the oracle uses, and compared with the
oracle on rough data, where the nonlinear weights are far from the ideal
ones and every constant of the closed forms matters.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from paper_2103_06080_amd import inputs as I


def _solve(A, b):
    """Exact Gauss-Jordan solve of a small square system over the rationals."""
    n = len(A)
    M = [list(row) + [bb] for row, bb in zip(A, b)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def _cell_average_row(j, deg):
    """Averages of x^p (p <= deg) over the unit cell [j - 1/2, j + 1/2]."""
    lo, hi = Fr(2 * j - 1, 2), Fr(2 * j + 1, 2)
    return [(hi ** (p + 1) - lo ** (p + 1)) / (p + 1) for p in range(deg + 1)]


def _poly_from_averages(offsets, values):
    """Coefficients c_p of the polynomial sum c_p x^p whose averages over the
    unit cells at the given offsets equal `values` (cell i is [-1/2, 1/2])."""
    deg = len(offsets) - 1
    return _solve([_cell_average_row(j, deg) for j in offsets], list(values))


def _peval(c, x):
    return sum(cp * x ** p for p, cp in enumerate(c))


def _pderiv(c):
    return [p * c[p] for p in range(1, len(c))]


def _pint_sq(c, lo, hi):
    """int_lo^hi (sum c_p x^p)^2 dx, exactly."""
    sq = [Fr(0)] * (2 * len(c) - 1)
    for a, ca in enumerate(c):
        for b, cb in enumerate(c):
            sq[a + b] += ca * cb
    return sum(s * (hi ** (p + 1) - lo ** (p + 1)) / (p + 1) for p, s in enumerate(sq))


STENCILS = {0: (-2, -1, 0), 1: (-1, 0, 1), 2: (0, 1, 2)}
HALF = Fr(1, 2)


def candidate(r, v5):
    """q_r and beta_r from the upwind-ordered values v5 = (v_{i-2}, .., v_{i+2})."""
    vals = [v5[j + 2] for j in STENCILS[r]]
    c = _poly_from_averages(STENCILS[r], vals)
    q = _peval(c, HALF)
    d1 = _pderiv(c)
    d2 = _pderiv(d1)
    # unit cells (dx = 1): the dx^(2l-1) factors and the derivative scalings cancel
    beta = _pint_sq(d1, -HALF, HALF) + _pint_sq(d2, -HALF, HALF)
    return q, beta


def ideal_weights():
    """d_r such that sum d_r q_r is the face value of the quartic through all
    five cell averages, for every choice of the averages."""
    basis = []
    for k in range(5):
        e = [Fr(0)] * 5
        e[k] = Fr(1)
        quartic = _peval(_poly_from_averages((-2, -1, 0, 1, 2), e), HALF)
        qs = [candidate(r, e)[0] for r in range(3)]
        basis.append((qs, quartic))
    # 5 equations sum_r d_r q_r(e_k) = quartic(e_k) in 3 unknowns (consistent)
    d = _solve([b[0] for b in basis[:3]], [b[1] for b in basis[:3]])
    for qs, quartic in basis:
        assert sum(dr * qr for dr, qr in zip(d, qs)) == quartic
    return d


D_IDEAL = None


def face_value(v5, eps):
    global D_IDEAL
    if D_IDEAL is None:
        D_IDEAL = ideal_weights()
    qs, a = [], []
    for r in range(3):
        q, beta = candidate(r, v5)
        qs.append(q)
        a.append(D_IDEAL[r] / (eps + beta) ** 2)
    s = sum(a)
    return sum(ar * qr for ar, qr in zip(a, qs)) / s, [ar / s for ar in a]


def exact_b(u, dtau, nl, alpha, eps):
    """b = -(F_{i+1/2} - F_{i-1/2}) / dtau with Lax-Friedrichs splitting
    f+- = (nl u^2/2 +- alpha u)/2: F+ reconstructed from the left on
    (i-2..i+2), F- from the right on the mirrored stencil (i+3..i-1)."""
    n = len(u)
    U = [Fr(float(x)) for x in u]
    nl, alpha, eps, dtau = Fr(nl), Fr(alpha), Fr(eps), Fr(dtau)
    fp = [(nl * x * x / 2 + alpha * x) / 2 for x in U]
    fm = [(nl * x * x / 2 - alpha * x) / 2 for x in U]
    F, W = [], []
    for i in range(n):
        vp = [fp[(i - 2 + r) % n] for r in range(5)]
        vm = [fm[(i + 3 - r) % n] for r in range(5)]
        Fp, wp = face_value(vp, eps)
        Fm, wm = face_value(vm, eps)
        F.append(Fp + Fm)
        W += [wp, wm]
    b = [-(F[i] - F[i - 1]) / dtau for i in range(n)]
    return np.array([float(x) for x in b]), W


def test_ideal_weights_from_the_quartic():
    """The linear weights that turn the three third-order candidates into the
    fifth-order value (the ideal weights of Jiang-Shu)."""
    assert ideal_weights() == [Fr(1, 10), Fr(6, 10), Fr(3, 10)]


def test_candidate_values_and_indicators_are_the_textbook_ones():
    """Sanity check of the exact construction itself on one stencil: q_1 and
    beta_1 of the centred candidate agree with the values for a quadratic
    whose averages are known by hand (p(x) = x^2: averages j^2 + 1/12)."""
    v5 = [Fr(j * j) + Fr(1, 12) for j in (-2, -1, 0, 1, 2)]
    for r in range(3):
        q, beta = candidate(r, v5)
        assert q == Fr(1, 4)                      # p(1/2) for every candidate
        assert beta == Fr(1, 3) + 4               # int (2x)^2 + int 2^2 over the unit cell


@pytest.mark.parametrize("seed,kind", [(1, "random"), (2, "random"), (3, "jumps"), (4, "spiky")])
def test_oracle_weno_b_equals_exact_rational_evaluation(orc, seed, kind):
    """The oracle's b on rough lines against the exact rational value (the
    only error left is the oracle's FP64 rounding).  The data are chosen so
    that the nonlinear weights are far from the ideal ones, where a wrong
    indicator constant, candidate coefficient or ideal weight changes b at
    O(1)."""
    n, dtau, nl = 24, 0.3, 0.8
    u = I.random_field(seed, (n,))
    if kind == "jumps":
        u = np.where(np.arange(n) % 7 < 3, 1.0, -0.4) + 0.05 * u
    elif kind == "spiky":
        u = 0.2 * u
        u[5] += 1.5
        u[13] -= 2.0
    alpha = abs(nl) * np.abs(u).max()
    eps = 1e-6
    ref, W = exact_b(u, dtau, nl, alpha, eps)
    got = orc.weno_b(u, dtau, nl, alpha, eps)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-13 * scale, np.abs(got - ref).max() / scale
    # the weights are far from ideal on a good share of the faces
    dev = [max(abs(float(w[r] - D_IDEAL[r])) for r in range(3)) for w in W]
    assert np.mean(np.array(dev) > 0.2) > 0.3


def test_oracle_weno_b_exact_on_smooth_data_too(orc):
    """Smooth data (weights near ideal): still the exact value to rounding."""
    n, L = 32, 8.0
    tau = -4 + L / n * np.arange(n)
    u = 0.5 + 0.25 * np.sin(2 * np.pi * tau / L)
    ref, _ = exact_b(u, L / n, 1.0, np.abs(u).max(), 1e-6)
    got = orc.weno_b(u, L / n, 1.0, np.abs(u).max(), 1e-6)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
