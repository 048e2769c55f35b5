"""kzk_step_noalloc (the march without device allocation, its memory in a
static per-GPU array) against kzk_step of a plan, through the C ABI: two
calls in a row on the same GPU, the second on a smaller input, each checked
against the plan-based march of the same problem (FP64 <= 1e-12, FP32 <=
1e-4 relative l2; the kernels are the same, so the fields are expected to
be equal bit for bit)."""
import numpy as np
import pytest

from paper_2103_06080_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-4}


def problem(nt, ny, n_steps, seed, scheduled):
    p = I.c1(n_steps=n_steps)
    p = I.Problem(**{**p.__dict__, "n_tau": nt, "n_y": ny})
    rng = I.SplitMix64(seed)
    T, a, modes = I._draw_nwave(rng)
    p.u0 = I.nwave(p.tau(), p.y(), T, a, 0.1, modes, p.y0, p.L_y)
    if scheduled:
        p.D_step = 0.05 * (1.0 + 0.3 * np.sin(np.arange(n_steps)))
        p.nl_node = 1.0 + 0.2 * np.cos(np.arange(n_steps + 1))
        p = I.Problem(**{**p.__dict__, "D_const": None, "nl_const": None})
    p.A = 1e-4
    return p


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_march_matches_plan_march(dtype):
    import torch
    from paper_2103_06080_amd import kzk
    assert torch.cuda.is_available()
    # the first call is the larger one: the second reuses memory holding the
    # first call's tables, state and status
    cases = [problem(1024, 512, 12, 1, True), problem(256, 64, 7, 2, False)]
    for p in cases:
        plan = kzk.Plan(p, dtype=dtype)
        ref = plan.pack([p.u0])
        plan.step(ref, 0, p.n_steps)
        assert plan.poll() == 0
        plan.close()
        u = torch.from_numpy(np.ascontiguousarray(p.u0).ravel()).to(
            device="cuda", dtype=torch.float32 if dtype == "f32" else torch.float64)
        st = kzk.step_noalloc(p, u, 0, p.n_steps, dtype=dtype)
        assert st == 0, st
        got = u.double().cpu().numpy().reshape(p.n_y, p.n_tau)
        want = ref.double().cpu().numpy().reshape(p.n_y, p.n_tau)
        err = rel_l2(got, want)
        print("noalloc %s %dx%d, %d steps: rel l2 vs plan %.2e, bitwise equal %s"
              % (dtype, p.n_tau, p.n_y, p.n_steps, err, np.array_equal(got, want)))
        assert err <= TOL[dtype]


def test_noalloc_rejects_what_does_not_fit():
    import torch
    from paper_2103_06080_amd import kzk
    p = problem(4096, 2048, 1, 3, False)          # 2^23 points: far above the array
    u = torch.zeros(p.points, dtype=torch.float32, device="cuda")
    assert kzk.step_noalloc(p, u, 0, 1, dtype="f32") == 2     # KZK_ERR_SIZE
    q = problem(64, 16, 3, 4, False)
    v = torch.from_numpy(q.u0.ravel().copy()).to("cuda")
    assert kzk.step_noalloc(q, v, 0, 3, dtype="f64") == 0     # still usable afterwards
