"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: FP64 GPU path <= 1e-12 relative l2 against the oracle, FP32 <= 1e-4
(per result), bit-exact where the result is exact (resume, invariant DC mode).
"""
import math

import numpy as np
import pytest

from paper_2103_06080_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-4}


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def small(nt, ny, n_steps=10, h=1e-3, D=0.05, nl=1.0, A=0.0, seed=0, amp=1.0):
    p = I.Problem(name="t", n_tau=nt, n_y=ny, h=h, n_steps=n_steps,
                  D_step=np.full(n_steps, float(D)), nl_node=np.full(n_steps + 1, float(nl)),
                  u0=np.zeros((ny, nt)), A=A, D_const=float(D), nl_const=float(nl))
    rng = I.SplitMix64(seed)
    T = rng.uniform_range(0.5, 1.5)
    p.u0 = I.nwave(p.tau(), p.y(), T, amp, 0.2, [(0.05, 1, 0.3), (0.03, 2, 1.0)], p.y0, p.L_y)
    return p


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nt,ny", [(32, 16), (256, 128), (8192, 16)])
def test_tau_transform_matches_rfft(torch_cuda, dtype, nt, ny):
    from paper_2103_06080_amd import kzk
    p = small(nt, ny)
    p.u0 = I.random_field(3, (ny, nt))
    plan = kzk.Plan(p, dtype=dtype)
    u = plan.pack([p.u0])
    spec = plan.tau_forward(u).double().cpu().numpy().reshape(ny, nt // 2, 2)
    spec = spec[..., 0] + 1j * spec[..., 1]
    ref = np.fft.rfft(p.u0, axis=1)
    got = spec.copy()
    assert np.allclose(got[:, 0].real, ref[:, 0].real, atol=1e-12 if dtype == "f64" else 1e-4)
    assert np.allclose(got[:, 0].imag, ref[:, nt // 2].real, atol=1e-12 if dtype == "f64" else 1e-4)
    tol = 1e-14 if dtype == "f64" else 1e-6
    assert rel_l2(got[:, 1:], ref[:, 1:nt // 2]) < tol * 10
    back = plan.tau_inverse(plan.tau_forward(u)).double().cpu().numpy().reshape(ny, nt)
    assert rel_l2(back, p.u0) < tol * 10


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nt,ny", [(64, 16), (256, 32), (2048, 16), (8192, 16)])
def test_weno_b_matches_oracle(torch_cuda, orc, dtype, nt, ny):
    from paper_2103_06080_amd import kzk
    p = small(nt, ny, nl=0.8)
    plan = kzk.Plan(p, dtype=dtype)
    b = plan.eval_b(plan.pack([p.u0]), 0).double().cpu().numpy().reshape(ny, nt)
    ref = np.stack([orc.weno_b(p.u0[j], p.dtau, 0.8, 0.8 * np.abs(p.u0[j]).max()) for j in range(ny)])
    # FP32: the round trip through the tau-transforms leaves ~1e-7 relative noise in u,
    # which the flux difference amplifies by ~max|u|/dtau (n_tau/8 here)
    assert rel_l2(b, ref) < (1e-12 if dtype == "f64" else max(2e-5, 2.5e-8 * nt))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shapes", [[(64, 16), (512, 32), (2048, 16), (256, 64)],
                                    [(512, 1024), (1024, 512), (4096, 128)]])
def test_weno_b_of_a_batched_plan_matches_oracle(torch_cuda, orc, dtype, shapes):
    """b of every solve of a plan of uneven grids: each solve's flux-difference
    symbols (its own n_tau and dtau) and tile layout; the second set has
    M >= 256 and M/16 >= W in every solve (progression-indexed tau-pass)."""
    from paper_2103_06080_amd import kzk
    probs = [small(nt, ny, nl=0.7, seed=i) for i, (nt, ny) in enumerate(shapes)]
    plan = kzk.Plan(probs, dtype=dtype)
    b = plan.eval_b(plan.pack([p.u0 for p in probs]), 0)
    for p, got in zip(probs, plan.unpack(b)):
        ref = np.stack([orc.weno_b(p.u0[j], p.dtau, 0.7, 0.7 * np.abs(p.u0[j]).max()) for j in range(p.n_y)])
        assert rel_l2(got, ref) < (1e-12 if dtype == "f64" else max(2e-5, 2.5e-8 * p.n_tau)), (p.n_tau, p.n_y)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nt,ny,n_steps,A", [(64, 16, 1, 0.0), (256, 128, 10, 1e-3), (128, 256, 5, 0.0),
                                             (512, 64, 7, 2e-4), (32, 4096, 2, 0.0), (8192, 32, 2, 1e-4),
                                             (512, 1024, 3, 1e-4), (2048, 1024, 2, 1e-4)])
def test_step_matches_oracle(torch_cuda, orc, dtype, nt, ny, n_steps, A):
    from paper_2103_06080_amd import kzk
    p = small(nt, ny, n_steps=n_steps, A=A)
    plan = kzk.Plan(p, dtype=dtype)
    u = plan.pack([p.u0])
    plan.step(u, 0, n_steps)
    assert plan.poll() == 0
    got = plan.unpack(u)[0]
    ref = orc.run(p)
    assert rel_l2(got, ref) < TOL[dtype], (rel_l2(got, ref))


@pytest.mark.parametrize("dtype,yt", [("f64", 256), ("f64", 512), ("f32", 256), ("f32", 512), ("f32", 1024)])
def test_full_tile_y_pass_matches_oracle(torch_cuda, orc, dtype, yt):
    """Grids whose y-tiles fill every thread slot (W n_y = 16 threads, n_y >= 512)
    take the full-tile y-pass; tau-lines of M >= 256 the progression-indexed
    pre/post-processing.  Coefficient schedules (D_step and nl_node, no
    constants): stage 1 evaluates the step's multipliers itself (FP64) and
    leaves h Phi2 for stage 2; each stage takes nl at its own node."""
    from paper_2103_06080_amd import kzk
    p = small(1024, 1024, n_steps=3, A=1e-4)
    p.D_step = 0.05 * (1.0 + 0.3 * np.sin(1.0 + np.arange(p.n_steps)))
    p.nl_node = 1.0 + 0.2 * np.cos(np.arange(p.n_steps + 1))
    p = I.Problem(**{**p.__dict__, "D_const": None, "nl_const": None})
    plan = kzk.Plan(p, dtype=dtype, y_threads=yt)
    assert plan.y_threads == yt
    u = plan.pack([p.u0])
    plan.step(u, 0, p.n_steps)
    assert plan.poll() == 0
    got = plan.unpack(u)[0]
    ref = orc.run(p)
    assert rel_l2(got, ref) < TOL[dtype], (rel_l2(got, ref))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c1_full_run_matches_oracle(torch_cuda, orc, dtype):
    from paper_2103_06080_amd import kzk
    p = I.c1()
    plan = kzk.Plan(p, dtype=dtype)
    u = plan.pack([p.u0])
    plan.step(u, 0, p.n_steps)
    assert plan.poll() == 0
    got = plan.unpack(u)[0]
    ref = orc.run(p)
    err = rel_l2(got, ref)
    print("c1 %s rel l2 = %.3e" % (dtype, err))
    assert err < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_runs_are_deterministic_and_resumable(torch_cuda, dtype):
    """Two identical marches agree bitwise (no atomics or races in the
    arithmetic); a march split in two agrees with the whole one up to the
    extra tau-transform round trip at the split."""
    from paper_2103_06080_amd import kzk
    p = small(256, 64, n_steps=12)
    plan = kzk.Plan(p, dtype=dtype)
    u1 = plan.pack([p.u0])
    plan.step(u1, 0, 12)
    u0 = plan.pack([p.u0])
    plan.step(u0, 0, 12)
    u2 = plan.pack([p.u0])
    plan.step(u2, 0, 5)
    plan.step(u2, 5, 7)
    assert plan.poll() == 0
    assert torch_cuda.equal(u1, u0)
    a, b = plan.unpack(u1)[0], plan.unpack(u2)[0]
    assert rel_l2(b, a) < (1e-14 if dtype == "f64" else 1e-6)


def test_status_nonfinite_and_cfl(torch_cuda):
    from paper_2103_06080_amd import kzk
    p = small(64, 16)
    plan = kzk.Plan(p, dtype="f64")
    u = plan.pack([p.u0])
    u[5] = float("nan")
    plan.step(u, 0, 1)
    assert plan.poll() == 6
    assert plan.poll() == 0          # cleared
    q = small(64, 16, h=0.5)         # alpha h / dtau = 0.5 * 1 / 0.125 = 4
    plan2 = kzk.Plan(q, dtype="f64", cfl_max=1.0)
    u = plan2.pack([q.u0])
    plan2.step(u, 0, 1)
    assert plan2.poll() == 5


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("h,A", [(1e-3, 0.0), (0.5, 2e-3)])
def test_multiplier_tables_match_oracle(torch_cuda, orc, dtype, h, A):
    """E, Phi1, Phi2 of z = h l(m, n), built on the GPU in FP64 (series near 0,
    closed forms elsewhere) and stored in the working precision, against the
    oracle's symbol and phi-functions; h = 0.5 reaches |z| ~ 2.5."""
    from paper_2103_06080_amd import kzk
    nt, ny = 64, 64
    p = small(nt, ny, h=h, A=A)
    plan = kzk.Plan(p, dtype=dtype)
    E, P1, P2 = plan.read_tables()
    M, Nh = nt // 2, ny // 2 + 1
    z = np.array([[h * orc.symbol(p, m, n, p.D_const) for n in range(Nh)] for m in range(M)])
    rE, r1, r2 = (orc.phi(k, z.ravel()).reshape(z.shape) for k in range(3))
    tol = 1e-14 if dtype == "f64" else 3e-7
    sl = (slice(1, None), slice(None))
    assert np.abs(E[sl] * ny - rE[sl]).max() < tol
    assert np.abs(P1[sl] * ny / h - r1[sl]).max() < tol
    assert np.abs(P2[sl] * ny / h - r2[sl]).max() < tol
    # tau-Nyquist scalars in slot (0, 0)
    zN = h * orc.symbol(p, M, 0, p.D_const)
    assert abs(E[0, 0] - orc.phi(0, zN)[0]) < tol
    assert abs(P1[0, 0] / h - orc.phi(1, zN)[0]) < tol
    assert abs(P2[0, 0] / h - orc.phi(2, zN)[0]) < tol
    if h == 0.5:
        assert np.abs(z).max() > 2.0 and np.abs(z[1:]).min() < 1.0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_stage1_phi2_of_a_scheduled_step_matches_oracle(torch_cuda, orc, dtype):
    """With an x-dependent D the first y-pass evaluates the step's multipliers
    itself and leaves h Phi2 / n_y in the table for the second; after a march
    of k steps that table holds Phi2 of step k-1's D (|z| up to ~1.9)."""
    from paper_2103_06080_amd import kzk
    nt, ny, k = 64, 64, 5
    p = small(nt, ny, n_steps=8, h=0.5, A=2e-3)
    p.D_step = 0.05 * (1 + 0.3 * np.sin(np.arange(p.n_steps)))
    p = I.Problem(**{**p.__dict__, "D_const": None, "nl_const": None})
    plan = kzk.Plan(p, dtype=dtype)
    u = plan.pack([p.u0 * 1e-3])
    plan.step(u, 0, k)
    assert plan.poll() == 0
    _, _, P2 = plan.read_tables()
    M, Nh = nt // 2, ny // 2 + 1
    Db = float(p.D_step[k - 1])
    z = np.array([[p.h * orc.symbol(p, m, n, Db) for n in range(Nh)] for m in range(M)])
    r2 = orc.phi(2, z.ravel()).reshape(z.shape)
    tol = 1e-14 if dtype == "f64" else 3e-7
    assert np.abs(P2[1:] * ny / p.h - r2[1:]).max() < tol
    zN = p.h * orc.symbol(p, M, 0, Db)
    assert abs(P2[0, 0] / p.h - orc.phi(2, zN)[0]) < tol
    assert np.abs(P2[0, 1:]).max() == 0
    assert np.abs(z).max() > 1.5    # both branches of the phi evaluation are used
