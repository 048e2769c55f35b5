"""Parity at the full sizes of the workloads, in the launch configuration the
benchmark times, through properties the oracle (or mathematics) can check:

* y-independent fields stay y-independent, so every row of the full 2D march
  must equal the oracle's 1D march of the same tau-profile (nonlinear WENO5
  part, absorption, coefficient schedules, table rebuild every step);
* with nl = 0 the march is exact for the linear part, so a cos(k tau) x
  Gaussian(y) field follows the closed form with c = s^2 - i (int D dx)/k
  (diffraction at full size, step-averaged D(x), absorption);
* the batched workload (64 uneven solves in one plan, graph replay) equals
  the same solves run one by one, bitwise.
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


def y_independent(p):
    """Same problem, initial field replaced by its seeded tau-profile (no y-modulation)."""
    rng = I.SplitMix64(0)
    T, a, _ = I._draw_nwave(rng)
    q = I.Problem(**{**p.__dict__})
    q.u0 = I.nwave(p.tau(), p.y(), T, a, 0.05, [], p.y0, p.L_y)
    return q


def one_row(p):
    q = I.Problem(**{**p.__dict__})
    q.n_y = 1
    q.u0 = p.u0[:1].copy()
    return q


@pytest.mark.parametrize("cfg", ["c3", "c2"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_full_march_of_y_independent_field_matches_oracle_line(torch_cuda, orc, cfg, dtype):
    from paper_2103_06080_amd import kzk
    p = y_independent({"c3": I.c3, "c2": I.c2}[cfg]())
    ref = orc.run(one_row(p))[0]
    plan = kzk.Plan(p, dtype=dtype)
    u = plan.pack([p.u0])
    plan.step(u, 0, p.n_steps)
    assert plan.poll() == 0
    got = plan.unpack(u)[0]
    rows = [0, 1, p.n_y // 3, p.n_y // 2, p.n_y - 1]
    err = max(rel_l2(got[j], ref) for j in rows)
    spread = float(np.abs(got - got[0:1]).max())
    print("%s %s full march (%d steps) y-independent: max row rel l2 %.3e, row spread %.1e"
          % (cfg, dtype, p.n_steps, err, spread))
    assert spread <= 1e-5 * np.abs(ref).max() if dtype == "f32" else spread <= 1e-13 * np.abs(ref).max()
    assert err < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_full_c3_linear_march_matches_closed_form(torch_cuda, dtype):
    from paper_2103_06080_amd import kzk
    p = I.c3()
    p.nl_node = np.zeros_like(p.nl_node)
    tau, y = p.tau(), p.y()
    k, s = 2 * math.pi * 3 / p.L_tau, 1.0
    p.u0 = np.cos(k * tau)[None, :] * np.exp(-y ** 2 / (2 * s * s))[:, None]
    plan = kzk.Plan(p, dtype=dtype)
    u = plan.pack([p.u0])
    plan.step(u, 0, p.n_steps)
    assert plan.poll() == 0
    got = plan.unpack(u)[0]
    X = p.h * p.n_steps
    intD = float(p.h * p.D_step.sum())
    c = s * s - 1j * intD / k
    ref = math.exp(-p.A * k * k * X) * np.real(
        np.exp(1j * k * tau)[None, :] * (s / np.sqrt(c)) * np.exp(-y ** 2 / (2 * c))[:, None])
    err = rel_l2(got, ref)
    print("c3 %s linear full march vs closed form: rel l2 %.3e" % (dtype, err))
    assert err < TOL[dtype]


def test_batched_small_solves_match_oracle(torch_cuda, orc):
    from paper_2103_06080_amd import kzk
    shapes = [(64, 16), (128, 32), (256, 64), (32, 128), (512, 16)]
    probs = []
    for i, (nt, ny) in enumerate(shapes):
        p = I.c1(n_steps=15)
        p = I.Problem(**{**p.__dict__, "n_tau": nt, "n_y": ny})
        rng = I.SplitMix64(i)
        T, a, modes = I._draw_nwave(rng)
        p.u0 = I.nwave(p.tau(), p.y(), T, a, 0.2, modes, p.y0, p.L_y)
        p.D_step = np.full(15, 0.01 + 0.01 * i)
        p.D_const = float(p.D_step[0])
        probs.append(p)
    for dtype in ("f64", "f32"):
        plan = kzk.Plan(probs, dtype=dtype)
        u = plan.pack([p.u0 for p in probs])
        plan.step(u, 0, 15)
        assert plan.poll() == 0
        for p, got in zip(probs, plan.unpack(u)):
            assert rel_l2(got, orc.run(p)) < TOL[dtype], (dtype, p.n_tau, p.n_y)


def test_c4_batched_graph_matches_single_solves(torch_cuda):
    """64 uneven solves, 500 steps, one plan, replayed through a HIP graph,
    equal bitwise to the same solves planned alone (same kernels and tiles)."""
    torch = torch_cuda
    from paper_2103_06080_amd import kzk
    probs = I.c4()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = kzk.Plan(probs, dtype="f32", stream=stream, graph=True)
        u0 = plan.pack([p.u0 for p in probs])
        u = u0.clone()
        plan.step(u, 0, 500)              # captured, then launched
        assert plan.poll() == 0
        first = u.clone()
        plan.set_graph(False)
        u2 = u0.clone()
        plan.step(u2, 0, 500)             # eager march between graph launches
        assert plan.poll() == 0
        plan.set_graph(True)
        for rep in range(2):
            u.copy_(u0)
            plan.step(u, 0, 500)          # capture once more, then replay the cached graph
            assert plan.poll() == 0
            assert torch.equal(u, first), rep
        stream.synchronize()
    assert torch.equal(first, u2)
    got = plan.unpack(u)
    for i in (0, 7, 21, 42, 63):
        single = kzk.Plan(probs[i], dtype="f32", y_threads=plan.y_threads)
        v = single.pack([probs[i].u0])
        single.step(v, 0, 500)
        assert single.poll() == 0
        assert np.array_equal(single.unpack(v)[0], got[i]), i


def test_graph_replays_match_eager(torch_cuda):
    torch = torch_cuda
    from paper_2103_06080_amd import kzk
    p = I.c1(n_steps=30)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        eager = kzk.Plan(p, dtype="f64", stream=stream)
        ref = eager.pack([p.u0])
        eager.step(ref, 0, 30)
        graph = kzk.Plan(p, dtype="f64", stream=stream, graph=True)
        for rep in range(4):
            u = graph.pack([p.u0])
            graph.step(u, 0, 30)
            assert graph.poll() == 0
            assert torch.equal(u, ref), rep
            ref2 = eager.pack([p.u0])          # eager work between replays
            eager.step(ref2, 0, 30)
            assert torch.equal(ref2, ref)
        stream.synchronize()


def test_graph_replay_needs_a_stream_of_its_own(torch_cuda):
    """The legacy default stream cannot be captured: with graphs on, a plan
    without a stream of its own rejects kzk_step (KZK_ERR_STATE) before
    enqueueing anything, and marches eagerly again once graphs are off."""
    from paper_2103_06080_amd import kzk
    p = I.c1(n_steps=5)
    plan = kzk.Plan(p, dtype="f64", stream=torch_cuda.cuda.default_stream(), graph=True)
    u = plan.pack([p.u0])
    before = u.clone()
    with pytest.raises(kzk.KZKError) as e:
        plan.step(u, 0, 5)
    assert e.value.code == 7
    assert plan.poll() == 0
    assert torch_cuda.equal(u, before)
    plan.set_graph(False)
    plan.step(u, 0, 5)
    assert plan.poll() == 0
    assert not torch_cuda.equal(u, before)
    plan.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_autotune_picks_a_supported_size_and_keeps_results(torch_cuda, orc, dtype):
    from paper_2103_06080_amd import kzk
    p = I.c1(n_steps=10)
    plan = kzk.Plan(p, dtype=dtype)
    u = plan.pack([p.u0])
    before = u.clone()
    best = plan.autotune(u, 3)
    assert best in ((1024, 512, 256) if dtype == "f32" else (512, 256))
    assert plan.y_threads == best
    import torch
    assert torch.equal(u, before)
    plan.step(u, 0, 10)
    assert plan.poll() == 0
    assert rel_l2(plan.unpack(u)[0], orc.run(p)) < TOL[dtype]


def test_autotune_cache_stores_and_reuses_the_choice(torch_cuda, orc, tmp_path, monkeypatch):
    """KZK_TUNE_CACHE: a timed result is appended as one line (key, y-pass
    threads, tau-pass threads, tau radix schedule, ms); a plan with the same
    key takes the last stored choice without timing."""
    from paper_2103_06080_amd import kzk
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("KZK_TUNE_CACHE", str(cache))
    p = I.c1(n_steps=6)
    plan = kzk.Plan(p, dtype="f32")
    u = plan.pack([p.u0])
    best = plan.autotune(u, 2)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    key, yt, tt, rx, ms = lines[0].split(" ")
    assert key.startswith("kzk2|") and (int(yt), int(tt), int(rx)) == tuple(plan.tuning().values())
    assert int(yt) == best and int(rx) in (8, 16) and float(ms) > 0
    plan.close()
    # a stored line for the same key wins (the last one), with no new timing
    with open(cache, "a") as f:
        f.write("%s 256 512 8 0.0100\n" % key)
    plan = kzk.Plan(p, dtype="f32")
    assert plan.autotune(u, 2) == 256
    assert plan.tuning() == {"y_threads": 256, "tau_threads": 512, "tau_fft_radix": 8}
    assert len(cache.read_text().splitlines()) == 2
    plan.step(u, 0, 6)
    assert plan.poll() == 0
    assert rel_l2(plan.unpack(u)[0], orc.run(p)) < TOL["f32"]
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nt,ny,tt", [(32, 64, 256), (64, 16, 256), (256, 128, 256), (2048, 64, 256),
                                      (8192, 16, 256), (1024, 1024, 512), (4096, 32, 512)])
def test_radix8_schedule_matches_radix16_and_oracle(torch_cuda, orc, dtype, nt, ny, tt):
    """The radix-8 tau-transform schedule (kzk_set_tau_fft_radix(8)) on every
    stage shape (tails of radix 2 and 4, the 2^12 = 8^4 transform, the
    progression-indexed pre/post-processing at 1024 x 1024, 512-thread blocks
    in FP32): the same march as the radix-16 schedule up to rounding, and the
    oracle's within the bars."""
    from paper_2103_06080_amd import kzk
    if dtype == "f64":
        tt = 256
    p = I.c1(n_steps=4)
    p = I.Problem(**{**p.__dict__, "n_tau": nt, "n_y": ny, "L_tau": 8.0, "tau0": -4.0, "h": 2e-4})
    rng = I.SplitMix64(11)
    T, a, modes = I._draw_nwave(rng)
    p.u0 = I.nwave(p.tau(), p.y(), T, a, 0.2, modes, p.y0, p.L_y)
    out = {}
    for r in (16, 8):
        plan = kzk.Plan(p, dtype=dtype, tau_threads=tt, tau_fft_radix=r)
        assert plan.tau_fft_radix == r
        u = plan.pack([p.u0])
        plan.step(u, 0, p.n_steps)
        assert plan.poll() == 0
        out[r] = plan.unpack(u)[0]
        plan.close()
    ref = orc.run(p)
    assert rel_l2(out[8], out[16]) < (1e-14 if dtype == "f64" else 2e-6)
    assert rel_l2(out[8], ref) < TOL[dtype]


def test_profile_sampling_counts_launches(torch_cuda):
    """kzk_profile_enable(k): the launches of every k-th step are bracketed
    (and the march's result does not depend on it)."""
    from paper_2103_06080_amd import kzk
    p = I.c1(n_steps=20)
    p = I.Problem(**{**p.__dict__, "D_const": None, "nl_const": None})   # per-step coefficients
    plan = kzk.Plan(p, dtype="f64")
    ref = plan.pack([p.u0])
    plan.step(ref, 0, 20)
    for every, n_prof in ((1, 20), (4, 5), (7, 3)):
        u = plan.pack([p.u0])
        plan.profile(True, every=every)
        plan.step(u, 0, 20)
        prof = plan.profile_read()
        plan.profile(False)
        assert prof["tau_pass"][1] == 2 * n_prof and prof["y_pass1"][1] == n_prof, (every, prof)
        assert prof["y_pass2"][1] == n_prof, (every, prof)
        assert torch_cuda.equal(u, ref)
    assert plan.poll() == 0
