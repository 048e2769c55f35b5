"""GPU parity on the paper's grid shape n_tau = N_theta = 7 2^k (Table 0, Sec. 4):
the mixed-radix tau-pass (a radix-7 Stockham stage, lines of M/16 threads in
groups of 2^(k-1), index wraps mod n_tau) against numpy's real FFT and the
FP64 oracle's mixed-radix transform, on every supported length 224 .. 7168,
with several lines per block and ragged last blocks, general and full-tile
y-passes, column tiles capped at the power of two dividing M, batched plans,
transport, the adjoint (also with 8192-row columns), and the full-size grids of sets 3 and 4 against the
closed form of the linear march and the oracle's march of a y-independent
field.

Bars: FP64 <= 1e-12 relative l2 (marches; 1e-14-level for transforms), FP32
<= 1e-4 for marches.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_2103_06080_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-4}
LENGTHS = [224, 448, 896, 1792, 3584, 7168]


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def small(nt, ny, n_steps=10, h=1e-3, D=0.05, nl=1.0, A=0.0, seed=0):
    p = I.Problem(name="g", n_tau=nt, n_y=ny, h=h, n_steps=n_steps,
                  D_step=np.full(n_steps, float(D)), nl_node=np.full(n_steps + 1, float(nl)),
                  u0=np.zeros((ny, nt)), A=A, D_const=float(D), nl_const=float(nl))
    rng = I.SplitMix64(seed)
    T = rng.uniform_range(0.5, 1.5)
    p.u0 = I.nwave(p.tau(), p.y(), T, 1.0, 0.2, [(0.05, 1, 0.3), (0.03, 2, 1.0)], p.y0, p.L_y)
    return p


def march(p, dtype, **kw):
    from paper_2103_06080_amd import kzk
    plan = kzk.Plan(p, dtype=dtype, **kw)
    u = plan.pack([p.u0])
    plan.step(u, 0, p.n_steps)
    assert plan.poll() == 0
    got = plan.unpack(u)[0]
    plan.close()
    return got


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nt", LENGTHS)
def test_tau_transform_of_7_2k_lines_matches_rfft(torch_cuda, orc, dtype, nt):
    from paper_2103_06080_amd import kzk
    ny = 16 if nt > 448 else 64
    p = small(nt, ny)
    p.u0 = I.random_field(5, (ny, nt))
    plan = kzk.Plan(p, dtype=dtype)
    u = plan.pack([p.u0])
    spec = plan.tau_forward(u).double().cpu().numpy().reshape(ny, nt // 2, 2)
    got = spec[..., 0] + 1j * spec[..., 1]
    ref = np.fft.rfft(p.u0, axis=1)
    # the oracle's own mixed-radix transform of one row agrees with numpy's
    row = p.u0[3]
    assert rel_l2(orc.fft(row.astype(complex))[:nt // 2 + 1], ref[3]) < 1e-13
    tol = 1e-14 if dtype == "f64" else 1e-6
    atol = 1e-12 if dtype == "f64" else 1e-4
    assert np.allclose(got[:, 0].real, ref[:, 0].real, atol=atol)
    assert np.allclose(got[:, 0].imag, ref[:, nt // 2].real, atol=atol)
    assert rel_l2(got[:, 1:], ref[:, 1:nt // 2]) < 10 * tol
    back = plan.tau_inverse(plan.tau_forward(u)).double().cpu().numpy().reshape(ny, nt)
    assert rel_l2(back, p.u0) < 10 * tol
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nt,ny", [(224, 16), (896, 32), (7168, 16)])
def test_weno_b_of_7_2k_lines_matches_oracle(torch_cuda, orc, dtype, nt, ny):
    from paper_2103_06080_amd import kzk
    p = small(nt, ny, nl=0.8)
    plan = kzk.Plan(p, dtype=dtype)
    b = plan.eval_b(plan.pack([p.u0]), 0).double().cpu().numpy().reshape(ny, nt)
    ref = np.stack([orc.weno_b(p.u0[j], p.dtau, 0.8, 0.8 * np.abs(p.u0[j]).max()) for j in range(ny)])
    assert rel_l2(b, ref) < (1e-12 if dtype == "f64" else max(2e-5, 2.5e-8 * nt))
    plan.close()


STEP_CASES = [
    # nt, ny, steps, A, y_threads
    (224, 64, 8, 0.0, None),
    (448, 128, 5, 1e-3, None),
    (448, 16, 4, 0.0, 256),       # tiles capped at 32 columns (the power of two dividing M = 224)
    (1792, 256, 3, 1e-4, None),
    (3584, 32, 2, 1e-4, None),
    (7168, 16, 2, 0.0, None),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", STEP_CASES, ids=["%dx%d" % (c[0], c[1]) + ("-yt%d" % c[4] if c[4] else "")
                                                  for c in STEP_CASES])
def test_march_on_7_2k_grid_matches_oracle(torch_cuda, orc, dtype, case):
    nt, ny, ns, A, yt = case
    p = small(nt, ny, n_steps=ns, A=A)
    got = march(p, dtype, y_threads=yt)
    ref = orc.run(p)
    err = rel_l2(got, ref)
    print("7 2^k march %s %s: rel l2 %.2e" % (dtype, case, err))
    assert err < TOL[dtype], err


@pytest.mark.parametrize("dtype,yt", [("f64", 512), ("f32", 1024), ("f32", 512)])
def test_full_tile_y_pass_on_7_2k_grid_matches_oracle(torch_cuda, orc, dtype, yt):
    """896 x 1024: tiles of 16 or 32 columns fill the y-pass block; coefficient
    schedules (stage 1 evaluates the multipliers), absorption."""
    p = small(896, 1024, n_steps=3, A=1e-4)
    p.D_step = 0.05 * (1.0 + 0.3 * np.sin(1.0 + np.arange(p.n_steps)))
    p.nl_node = 1.0 + 0.2 * np.cos(np.arange(p.n_steps + 1))
    p = dataclasses.replace(p, D_const=None, nl_const=None)
    got = march(p, dtype, y_threads=yt)
    ref = orc.run(p)
    assert rel_l2(got, ref) < TOL[dtype], rel_l2(got, ref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batched_7_2k_plan_matches_oracle(torch_cuda, orc, dtype):
    """Solves of one n_tau = 448 and uneven n_y in one plan."""
    from paper_2103_06080_amd import kzk
    probs = [small(448, ny, n_steps=4, A=2e-4, seed=i) for i, ny in enumerate((64, 256, 16))]
    plan = kzk.Plan(probs, dtype=dtype)
    u = plan.pack([q.u0 for q in probs])
    plan.step(u, 0, 4)
    assert plan.poll() == 0
    for q, got in zip(probs, plan.unpack(u)):
        assert rel_l2(got, orc.run(q)) < TOL[dtype], q.n_y
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scheme,reg", [(0, False), (1, True)])
def test_transport_on_7_2k_grid_matches_oracle(torch_cuda, orc, dtype, scheme, reg):
    """The full b (random velocity field) with n_tau = 7 2^k: both schemes,
    the plain and the regularised multiplier."""
    eps = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}[dtype]
    p = I.Problem(name="m", n_tau=448, n_y=64, h=2e-3, n_steps=6, D_step=np.full(6, 0.05),
                  nl_node=np.full(7, 0.9), u0=np.zeros((64, 448)), A=1e-4, D_const=0.05, nl_const=0.9,
                  x0=1.5, scheme=scheme, reg_eps=eps if reg else 0.0, **I.medium(7, 200))
    rng = I.SplitMix64(7)
    T, a, modes = I._draw_nwave(rng)
    p.u0 = I.nwave(p.tau(), p.y(), T, a, 0.1, modes, p.y0, p.L_y) + 0.1
    got = march(p, dtype)
    ref = orc.run(p)
    err = rel_l2(got, ref)
    print("7 2^k transport %s scheme %d reg %s: rel l2 %.2e" % (dtype, scheme, reg, err))
    assert err < TOL[dtype], err


def test_7_2k_plan_rejects_wide_tau_blocks(torch_cuda):
    from paper_2103_06080_amd import kzk
    p = small(448, 64, n_steps=2)
    plan = kzk.Plan(p, dtype="f32")
    assert plan.tau_threads == 256
    with pytest.raises(kzk.KZKError):
        plan.set_tau_threads(512)
    with pytest.raises(kzk.KZKError):
        plan.set_tau_fft_radix(8)
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nt,ny,n_steps,ckpt,scheduled", [(448, 32, 5, 2, True), (224, 64, 6, 3, False),
                                                         (1792, 16, 3, 3, True)])
def test_adjoint_on_7_2k_grid_matches_oracle(torch_cuda, orc, dtype, nt, ny, n_steps, ckpt, scheduled):
    """The discrete adjoint with the mixed-radix tau-transforms (the adjoint
    tau-pass in its 7 2^k form) against the oracle's adjoint."""
    from paper_2103_06080_amd import kzk
    from test_gpu_adjoint import nwave_problem
    p = nwave_problem(nt, ny, n_steps, scheduled=scheduled)
    lam = I.random_field(77, (ny, nt))
    ref = orc.adjoint(p, lam, ckpt=ckpt)
    plan = kzk.Plan(p, dtype=dtype)
    g = plan.adjoint(plan.pack([p.u0]), plan.pack([lam]), 0, n_steps, ckpt)
    assert plan.poll() == 0
    err = rel_l2(plan.unpack(g)[0], ref)
    print("7 2^k adjoint %s %dx%d %d steps: rel l2 %.3e" % (dtype, nt, ny, n_steps, err))
    assert err < (1e-12 if dtype == "f64" else 1e-4)
    plan.close()


def set3_linear(A=3.4e-4):
    """Set 3's grid and coefficients (1792 x 4096, Sigma = 120 in 1200 steps,
    D/2 = 1/(4 pi), absorption A) without the nonlinear term and the medium."""
    q = I.paper_set(3)
    return I.Problem(name="set3-linear", n_tau=q.n_tau, n_y=q.n_y, h=q.h, n_steps=q.n_steps,
                     D_step=q.D_step, nl_node=np.zeros_like(q.nl_node), u0=q.u0, tau0=q.tau0, L_tau=q.L_tau,
                     y0=q.y0, L_y=q.L_y, A=A, D_const=q.D_const, nl_const=0.0)


@pytest.mark.parametrize("dtype,state64,bar", [("f64", False, 1e-11), ("f32", True, 2e-5)])
def test_set3_grid_full_linear_march_matches_closed_form(torch_cuda, dtype, state64, bar):
    """u0 = cos(k tau) exp(-(y - y_c)^2 / (2 s^2)), one tau-mode: the march of
    u_x = D/2 ... solves exactly (the paper's linear part, eq. (20) with b = 0)
    to exp(-A k^2 X) Re[e^{i k tau} (s / sqrt(c)) exp(-(y - y_c)^2 / (2 c))],
    c = s^2 - i D X / k, as long as the Gaussian stays inside the period."""
    p = set3_linear()
    tau, y = p.tau(), p.y()
    k, s, yc = 2 * math.pi * 5 / p.L_tau, 12.0, 200.0
    p.u0 = np.cos(k * tau)[None, :] * np.exp(-(y - yc) ** 2 / (2 * s * s))[:, None]
    X = p.h * p.n_steps
    c = s * s - 1j * float(p.h * p.D_step.sum()) / k
    ref = math.exp(-p.A * k * k * X) * np.real(
        np.exp(1j * k * tau)[None, :] * (s / np.sqrt(c)) * np.exp(-(y - yc) ** 2 / (2 * c))[:, None])
    kw = {"state_fp64": True} if state64 else {}
    err = rel_l2(march(p, dtype, **kw), ref)
    print("set 3 grid (1792 x 4096) linear 1200-step march %s: rel l2 %.3e" % (dtype, err))
    assert err < bar, err


@pytest.mark.parametrize("dtype,bar", [("f64", 1e-11), ("f32", 1e-4)])
def test_set3_grid_full_march_of_y_independent_field_matches_oracle_line(torch_cuda, orc, dtype, bar):
    """Set 3's grid, coefficients, regularised multiplier and N-wave without
    the medium (the N-wave is y-independent, so every row marches like the
    oracle's single line): all 1200 steps to Sigma = 120."""
    eps = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}[dtype]
    q = I.paper_set(3, reg_eps=eps)
    p = I.Problem(name="set3-line", n_tau=q.n_tau, n_y=q.n_y, h=q.h, n_steps=q.n_steps, D_step=q.D_step,
                  nl_node=q.nl_node, u0=q.u0, tau0=q.tau0, L_tau=q.L_tau, y0=q.y0, L_y=q.L_y, A=q.A,
                  D_const=q.D_const, nl_const=q.nl_const, reg_eps=eps)
    line = dataclasses.replace(p, n_y=1, u0=p.u0[:1].copy())
    ref = orc.run(line)[0]
    got = march(p, dtype)
    err = max(rel_l2(got[j], ref) for j in (0, 1234, p.n_y - 1))
    print("set 3 grid y-independent 1200-step march %s: rel l2 %.3e" % (dtype, err))
    assert err < bar, err


# ---- 8192 rows (set 4 of Table 0: N_rho = 10000 -> n_y = 8192)

@pytest.mark.parametrize("dtype,yt", [("f64", 512), ("f32", 1024), ("f32", 512)])
@pytest.mark.parametrize("nt", [32, 448])
def test_march_with_8192_rows_matches_oracle(torch_cuda, orc, dtype, yt, nt):
    """Column transforms of 8192 points (twiddles loaded per stage) in the
    full-tile y-passes of 1 or 2 columns, with coefficient schedules."""
    p = small(nt, 8192, n_steps=3, A=1e-4)
    p.D_step = 0.05 * (1.0 + 0.3 * np.sin(1.0 + np.arange(p.n_steps)))
    p = dataclasses.replace(p, D_const=None)
    got = march(p, dtype, y_threads=yt)
    ref = orc.run(p)
    err = rel_l2(got, ref)
    print("8192 rows %s %d x 8192 (%d threads): rel l2 %.2e" % (dtype, nt, yt, err))
    assert err < TOL[dtype], err


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_transport_with_8192_rows_matches_oracle(torch_cuda, orc, dtype):
    """The full b and the regularised multiplier (mean column transformed along
    8192 rows) on a 64 x 8192 grid."""
    eps = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}[dtype]
    p = I.Problem(name="m", n_tau=64, n_y=8192, h=2e-3, n_steps=3, D_step=np.full(3, 0.05),
                  nl_node=np.full(4, 0.9), u0=np.zeros((8192, 64)), A=1e-4, D_const=0.05, nl_const=0.9,
                  x0=1.5, L_y=400.0, y0=0.0, reg_eps=eps, **I.medium(9, 200))
    rng = I.SplitMix64(9)
    T, a, modes = I._draw_nwave(rng)
    p.u0 = I.nwave(p.tau(), p.y(), T, a, 0.1, modes, p.y0, p.L_y) + 0.1
    got = march(p, dtype)
    ref = orc.run(p)
    err = rel_l2(got, ref)
    print("8192 rows transport %s: rel l2 %.2e" % (dtype, err))
    assert err < TOL[dtype], err


@pytest.mark.parametrize("dtype,yt,nt,n_steps", [("f64", 512, 32, 3), ("f32", 1024, 32, 3), ("f32", 512, 32, 3),
                                                  ("f64", 512, 448, 2)])
def test_adjoint_with_8192_rows_matches_oracle(torch_cuda, orc, dtype, yt, nt, n_steps):
    """The discrete adjoint with 8192-point column transforms (twiddles
    loaded per transform stage in both adjoint y-passes), in full tiles of
    1 or 2 columns, against the oracle's adjoint; on 448 x 8192 with the
    mixed-radix adjoint tau-pass as well."""
    from paper_2103_06080_amd import kzk
    from test_gpu_adjoint import nwave_problem
    p = nwave_problem(nt, 8192, n_steps, scheduled=True)
    lam = I.random_field(77, (8192, nt))
    ref = orc.adjoint(p, lam, ckpt=1)
    plan = kzk.Plan(p, dtype=dtype, y_threads=yt)
    g = plan.adjoint(plan.pack([p.u0]), plan.pack([lam]), 0, n_steps, 2)
    assert plan.poll() == 0
    err = rel_l2(plan.unpack(g)[0], ref)
    print("8192-row adjoint %s %d x 8192 (%d threads): rel l2 %.3e" % (dtype, nt, yt, err))
    assert err < (1e-12 if dtype == "f64" else 1e-4)
    plan.close()


def test_8192_rows_need_full_tiles_of_512_threads(torch_cuda):
    from paper_2103_06080_amd import kzk
    p = small(32, 8192, n_steps=2)
    plan = kzk.Plan(p, dtype="f32")
    assert plan.y_threads == 1024
    with pytest.raises(kzk.KZKError):
        plan.set_y_threads(256)
    plan.set_y_threads(512)
    assert plan.y_threads == 512
    plan.close()
    # a solve with few rows next to the 8192-row one leaves no full-tile layout
    with pytest.raises(kzk.KZKError):
        kzk.Plan([small(448, 8192, n_steps=2), small(448, 64, n_steps=2)], dtype="f32")


@pytest.mark.parametrize("dtype,state64,bar", [("f64", False, 1e-11), ("f32", True, 2e-5)])
def test_set4_grid_full_linear_march_matches_closed_form(torch_cuda, dtype, state64, bar):
    """Set 4's grid (3584 x 8192) and coefficients over its 2400 steps
    (Sigma = 120), nonlinear term and medium off, against the closed form."""
    q = I.paper_set(4)
    p = I.Problem(name="set4-linear", n_tau=q.n_tau, n_y=q.n_y, h=q.h, n_steps=q.n_steps, D_step=q.D_step,
                  nl_node=np.zeros_like(q.nl_node), u0=q.u0, tau0=q.tau0, L_tau=q.L_tau, y0=q.y0, L_y=q.L_y,
                  A=q.A, D_const=q.D_const, nl_const=0.0)
    tau, y = p.tau(), p.y()
    k, s, yc = 2 * math.pi * 5 / p.L_tau, 12.0, 200.0
    p.u0 = np.cos(k * tau)[None, :] * np.exp(-(y - yc) ** 2 / (2 * s * s))[:, None]
    X = p.h * p.n_steps
    c = s * s - 1j * float(p.h * p.D_step.sum()) / k
    ref = math.exp(-p.A * k * k * X) * np.real(
        np.exp(1j * k * tau)[None, :] * (s / np.sqrt(c)) * np.exp(-(y - yc) ** 2 / (2 * c))[:, None])
    kw = {"state_fp64": True} if state64 else {}
    err = rel_l2(march(p, dtype, **kw), ref)
    print("set 4 grid (3584 x 8192) linear 2400-step march %s: rel l2 %.3e" % (dtype, err))
    assert err < bar, err


@pytest.mark.parametrize("dtype,bar", [("f64", 1e-11), ("f32", 1e-4)])
def test_set4_grid_full_march_of_y_independent_field_matches_oracle_line(torch_cuda, orc, dtype, bar):
    """Set 4's grid, coefficients, regularised multiplier and N-wave without
    the medium: all 2400 steps against the oracle's single line."""
    eps = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}[dtype]
    q = I.paper_set(4, reg_eps=eps)
    p = I.Problem(name="set4-line", n_tau=q.n_tau, n_y=q.n_y, h=q.h, n_steps=q.n_steps, D_step=q.D_step,
                  nl_node=q.nl_node, u0=q.u0, tau0=q.tau0, L_tau=q.L_tau, y0=q.y0, L_y=q.L_y, A=q.A,
                  D_const=q.D_const, nl_const=q.nl_const, reg_eps=eps)
    line = dataclasses.replace(p, n_y=1, u0=p.u0[:1].copy())
    ref = orc.run(line)[0]
    got = march(p, dtype)
    err = max(rel_l2(got[j], ref) for j in (0, 4321, p.n_y - 1))
    print("set 4 grid y-independent 2400-step march %s: rel l2 %.3e" % (dtype, err))
    assert err < bar, err


@pytest.mark.parametrize("dtype,bar", [("f64", 1e-12), ("f32", 1e-4)])
def test_largest_grid_march_of_y_independent_field_matches_oracle_line(torch_cuda, orc, dtype, bar):
    """The largest supported grid, 8192 x 8192 (both transforms at their
    maximum length, 8192-row columns in full tiles), 20 steps of a nonlinear,
    absorbing march of a y-independent N-wave against the oracle's line."""
    p = small(8192, 8192, n_steps=20, h=2e-4, A=1e-4)
    p.u0 = np.tile(p.u0[:1], (8192, 1))
    line = dataclasses.replace(p, n_y=1, u0=p.u0[:1].copy())
    ref = orc.run(line)[0]
    got = march(p, dtype)
    err = max(rel_l2(got[j], ref) for j in (0, 5000, 8191))
    print("8192 x 8192 y-independent 20-step march %s: rel l2 %.2e" % (dtype, err))
    assert err < bar, err


def test_autotune_of_a_7_2k_plan_keeps_its_single_tau_layout(torch_cuda, orc):
    """The autotuner tries only the tau-pass block and radix schedule a
    7 2^k plan has (256 threads, radix-16 stages after the radix-7 one) and
    still picks among the y-pass layouts; the tuned march matches the oracle."""
    from paper_2103_06080_amd import kzk
    p = small(448, 128, n_steps=4, A=1e-4)
    plan = kzk.Plan(p, dtype="f32")
    u = plan.pack([p.u0])
    best = plan.autotune(u, 2)
    tun = plan.tuning()
    assert tun["tau_threads"] == 256 and tun["tau_fft_radix"] == 16 and tun["y_threads"] == best
    plan.step(u, 0, p.n_steps)
    assert plan.poll() == 0
    assert rel_l2(plan.unpack(u)[0], orc.run(p)) < TOL["f32"]
    plan.close()
