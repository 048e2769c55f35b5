"""GPU parity of the method variants with the FP64 oracle: exponential Euler
(Sec. 3.3) and the regularised Fourier multiplier (Sec. 3.4, definition of
z_jk), alone and together, on fields whose rows carry a y-dependent tau-mean
(so the mean tau-mode column is exercised), with constant and scheduled
coefficients, on general and full-tile y-passes.

Bars: FP64 <= 1e-12 relative l2, FP32 <= 1e-4 (and the largest pointwise
error <= the same factor times max|u|).
"""
import dataclasses

import numpy as np
import pytest

from paper_2103_06080_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-4}
EPS = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def problem(nt, ny, n_steps, h=1e-3, scheduled=False, seed=0):
    p = I.Problem(name="v", n_tau=nt, n_y=ny, h=h, n_steps=n_steps,
                  D_step=np.full(n_steps, 0.05), nl_node=np.full(n_steps + 1, 1.0),
                  u0=np.zeros((ny, nt)), A=1e-4, D_const=0.05, nl_const=1.0)
    rng = I.SplitMix64(seed)
    T, a, modes = I._draw_nwave(rng)
    y = p.y()
    mean = 0.2 + 0.1 * np.cos(2 * np.pi * (y - p.y0) / p.L_y) + 0.05 * np.sin(6 * np.pi * (y - p.y0) / p.L_y)
    p.u0 = I.nwave(p.tau(), y, T, a, 0.1, modes, p.y0, p.L_y) + mean[:, None]
    if scheduled:
        p.D_step = 0.05 * (1.0 + 0.3 * np.sin(1.0 + np.arange(n_steps)))
        p.nl_node = 1.0 + 0.2 * np.cos(np.arange(n_steps + 1))
        p = dataclasses.replace(p, D_const=None, nl_const=None)
    return p


def run_gpu(p, dtype, y_threads=None):
    from paper_2103_06080_amd import kzk
    plan = kzk.Plan(p, dtype=dtype, y_threads=y_threads)
    u = plan.pack([p.u0])
    plan.step(u, 0, p.n_steps)
    assert plan.poll() == 0
    got = plan.unpack(u)[0]
    plan.close()
    return got


CASES = [
    # (nt, ny, steps, h, scheduled, y_threads)
    (256, 64, 12, 1e-3, False, None),
    (512, 128, 8, 1e-3, True, None),
    (1024, 1024, 3, 1e-3, True, 512),     # full-tile y-pass, multipliers evaluated in stage 1
    (128, 256, 10, 2e-6, False, None),    # small step: the mean-mode multipliers of eps = 2^-24 are in (0, 1)
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scheme,reg", [(1, False), (0, True), (1, True)])
@pytest.mark.parametrize("case", CASES, ids=["%dx%d" % c[:2] + ("s" if c[4] else "") + ("h" if c[3] < 1e-4 else "")
                                             for c in CASES])
def test_variant_march_matches_oracle(torch_cuda, orc, dtype, scheme, reg, case):
    nt, ny, ns, h, sched, yt = case
    p = problem(nt, ny, ns, h, sched)
    p = dataclasses.replace(p, scheme=scheme, reg_eps=EPS[dtype] if reg else 0.0)
    ref = orc.run(p)
    got = run_gpu(p, dtype, yt)
    e2, em = rel_l2(got, ref), max_rel(got, ref)
    print("%s scheme %d reg %s %dx%d: rel l2 %.2e max %.2e" % (dtype, scheme, reg, nt, ny, e2, em))
    assert e2 < TOL[dtype] and em < TOL[dtype], (e2, em)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_regularised_mean_column_is_projected(torch_cuda, dtype):
    """eps = machine epsilon and an ordinary step: after one step every row has
    the y-averaged tau-mean (E_0 = 0 for ky != 0), unlike the unregularised
    method, which keeps each row's mean."""
    p = problem(256, 64, 1)
    p = dataclasses.replace(p, nl_node=np.zeros(2), nl_const=0.0)
    means0 = p.u0.mean(axis=1)
    kept = run_gpu(p, dtype)
    reg = run_gpu(dataclasses.replace(p, reg_eps=EPS[dtype]), dtype)
    tol = 1e-13 if dtype == "f64" else 1e-6
    assert np.abs(kept.mean(axis=1) - means0).max() < tol
    assert np.abs(reg.mean(axis=1) - means0.mean()).max() < tol


def test_adjoint_rejects_the_variants(torch_cuda):
    from paper_2103_06080_amd import kzk
    for kw in (dict(scheme=1), dict(reg_eps=1e-16)):
        p = dataclasses.replace(problem(64, 16, 2), **kw)
        plan = kzk.Plan(p, dtype="f64")
        u = plan.pack([p.u0])
        with pytest.raises(kzk.KZKError) as e:
            plan.adjoint(u, u.clone(), 0, 2, 1)
        assert e.value.code == 1
