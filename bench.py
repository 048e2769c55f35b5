#!/usr/bin/env python3
"""Throughput of the exponential-integrator/WENO5 march on one MI355X.

One bench "step" is one pass of the whole hot path over one batch of
synthetic input: the full inhomogeneous-medium march of an 8192 x 4096
(tau x y) N-wave, 2000 ExpRK22 steps with x-dependent nl(x), D(x) and
absorption, in FP32 (the FP64 multipliers of each step evaluated in the first y-pass).
Every bench step is that march from its initial field (x from 0 to 0.5),
copied from a resident copy in HBM, so every timed step does identical work.

Prints one JSON line: value = grid-point-steps per second, plus the
roofline of the dominant kernel (per-kernel HIP events over the timed
region), the error against the FP64 oracle (first steps of the workload on
the whole field; the full march on the stored oracle rows) and the FP64 CPU
oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
PROFILE_EVERY = 8              # per-kernel HIP events on every 8th step of the timed marches
# MI355X published vector peaks (FP32 counts packed FP32 instructions)
ALU_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
# issue rate of the instructions this build uses (no packed FP32):
# 256 CU x 64 lanes x 2 flops (FMA) x 2.4 GHz, the same in FP32 and FP64
NONPACKED_PEAK_TFLOPS = 78.6
ORACLE_STEPS = 8               # steps of the oracle sample (CPU baseline and first-steps parity)

WORKLOADS = {
    # name: (builder, default dtype)
    "c3": "inhomogeneous medium, 8192 x 4096, 2000 steps, h = 2.5e-4, A = 1e-4",
    "c2": "homogeneous medium, 4096 x 2048, 1000 steps, h = 5e-4",
    "c1": "plain method, 256 x 128, 200 steps, h = 1e-3",
    "c5": "adjoint workload's forward march, 2048 x 1024, 500 steps, h = 5e-4",
}
# (the 64-solve batched workload is measured in the side legs of the c3 run)


def kernel_model(kind, n_tau, n_y, esz):
    """Algorithmic bytes and flops of one launch (see the design notes):
    arrays are n_tau * n_y reals (the packed half-spectrum has the same size)."""
    N = n_tau * n_y
    arr = esz * N
    lg = (n_tau.bit_length() - 1)
    if kind == "tau_pass":
        # read C~, write B~; two real tau-FFTs (2.5 N log2 N each) + WENO5 (~120 flops/point)
        return 2 * arr, N * (5.0 * lg + 120.0)
    if kind == "y_pass1":
        # read B~, U; write P, C~*; two complex y-FFTs of N/2 points + combine
        lgy = (n_y.bit_length() - 1)
        return 4 * arr, N * (2 * 2.5 * lgy + 12.0)
    if kind == "y_pass2":
        # read B~*, P; write U, C~
        lgy = (n_y.bit_length() - 1)
        return 4 * arr, N * (2 * 2.5 * lgy + 4.0)
    return None, None


def kernel_source_sha():
    """sha256 over the device sources (kernels, FFT stages, shared descriptors)."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "fft.hpp", "internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2103_06080_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def pmc_traffic(kernel_kind, workload, dtype):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s_%s.json" % (kernel_kind, workload, dtype))
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        if rec.get("kernels_sha256") != kernel_source_sha():
            return None
        return rec.get("hbm_bytes_per_launch")
    except Exception:
        return None


def cpu_baseline(problem, n_steps=ORACLE_STEPS):
    """The FP64 oracle, as it stands, on the first n_steps ExpRK22 steps of the
    same workload; the rate counts the step loop only (each step with its
    FP64 multiplier build), not the transforms at the ends of the run.
    Returns the record and the oracle's field after the steps."""
    from oracle import oracle
    oracle.lib()
    t0 = time.perf_counter()
    ref = oracle.run(problem, n_steps=n_steps)
    total = time.perf_counter() - t0
    dt = oracle.last_step_seconds()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rec = {"value": problem.points * n_steps / dt, "unit": "grid-point-steps/s", "cores": cores, "kind": "oracle",
           "sample": "the first %d ExpRK22 steps of the %d x %d workload (its FP64 multipliers rebuilt every "
                     "step); step loop %.1f s of a %.1f s run that also holds the two 2D transforms"
                     % (n_steps, problem.n_tau, problem.n_y, dt, total)}
    return rec, ref


def rel_l2(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def first_steps_error(problem, ref, dtype, n_steps=ORACLE_STEPS):
    """GPU march of the same first steps against the oracle's (rel. l2 over
    the field, and the largest pointwise error over max|u|)."""
    import numpy as np
    from paper_2103_06080_amd import kzk
    plan = kzk.Plan(problem, dtype=dtype)
    u = plan.pack([problem.u0])
    plan.step(u, 0, n_steps)
    assert plan.poll() == 0
    got = plan.unpack(u)[0]
    plan.close()
    return {"steps": n_steps, "rel_l2": rel_l2(got, ref),
            "max_err_over_max_u": float(np.abs(got - ref).max() / np.abs(ref).max())}


def sampled_march_error(name, u_host, n_steps):
    """Rows of a full march against the stored oracle rows of the same march
    (tests/golden, written by a script that calls only the oracle)."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "%s_seed0_oracle_rows.npz" % name)
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    key = "u_step%d" % n_steps
    if key not in z.files:
        return None
    rows = z["rows_final"]
    ref = z[key]
    got = u_host[rows]
    return {"steps": n_steps, "rows": len(rows), "of_rows": int(u_host.shape[0]), "rel_l2": rel_l2(got, ref),
            "max_err_over_max_u": float(np.abs(got - ref).max() / np.abs(ref).max())}


def measured_copy_gbs(mib=1024, reps=5):
    """Device-to-device copy bandwidth (bytes read + written per second) of a
    mib-MiB buffer, the best of reps copies timed with events."""
    import torch
    src = torch.ones(mib * (1 << 18), dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * mib * (1 << 20) / best / 1e9


def _time(fn, sync):
    sync()
    t0 = time.perf_counter()
    fn()
    sync()
    return time.perf_counter() - t0


def progress(msg):
    """One line on stderr as each leg of the benchmark ends."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def side_measurements(args, value_fp32, ms_fp32):
    """FP64 march of the same workload, the adjoint/forward time ratio on the
    2048 x 1024 adjoint workload, and the batched 64-solve throughput."""
    import torch
    from paper_2103_06080_amd import inputs, kzk
    sync = torch.cuda.synchronize
    out = {}
    # FP64, the same march (steps 0 .. 1999 from the initial field)
    p = inputs.c3()
    plan = kzk.Plan(p, dtype="f64")
    u0 = plan.pack([p.u0])
    u = u0.clone()
    plan.step(u, 0, p.n_steps)

    def fp64_march():
        u.copy_(u0)
        plan.step(u, 0, p.n_steps)
    t = _time(fp64_march, sync)
    assert plan.poll() == 0
    v64 = p.points * p.n_steps / t
    out["fp64_c3"] = {"s_per_march": t, "value": v64, "fp32_speedup": value_fp32 / v64,
                      "y_threads": plan.y_threads}
    progress("FP64 march done")
    plan.close()
    del plan, u, u0
    torch.cuda.empty_cache()
    # FP32 with the spectral state in FP64: the same march, its error on the
    # stored oracle rows, and the error of the linear 2000-step march against
    # its closed form (plain FP32 state and FP64 state)
    plan = kzk.Plan(p, dtype="f32", state_fp64=True)
    u0 = plan.pack([p.u0])
    u = u0.clone()
    plan.step(u, 0, p.n_steps)

    def s64_march():
        u.copy_(u0)
        plan.step(u, 0, p.n_steps)
    t = _time(s64_march, sync)
    assert plan.poll() == 0
    rows = sampled_march_error("c3", u.double().cpu().numpy().reshape(p.n_y, p.n_tau), p.n_steps)
    plan.close()
    del plan, u, u0
    torch.cuda.empty_cache()
    out["fp32_state64_c3"] = {"s_per_march": t, "value": p.points * p.n_steps / t,
                              "slowdown_vs_fp32_state": t / (p.points * p.n_steps / value_fp32),
                              "full_march_sampled_rows": rows,
                              "linear_march_vs_closed_form": {"fp32_state": linear_march_error(False),
                                                              "fp64_state": linear_march_error(True)}}
    progress("FP32 march with FP64 state done")
    # adjoint / forward on the adjoint workload (FP32 and FP64); its 8 / 16 MB
    # arrays fit the 256 MB Infinity Cache, so these rates are cache-assisted
    q = inputs.c5()
    for dt in ("f32", "f64"):
        plan = kzk.Plan(q, dtype=dt)
        u0 = plan.pack([q.u0])
        u = u0.clone()
        plan.step(u, 0, q.n_steps)
        u.copy_(u0)
        tf = _time(lambda: plan.step(u, 0, q.n_steps), sync)
        lam = torch.ones_like(u0)
        plan.adjoint(u0, lam, 0, q.n_steps, inputs.C5_CKPT)
        ta = _time(lambda: plan.adjoint(u0, lam, 0, q.n_steps, inputs.C5_CKPT), sync)
        # one segment (checkpoint interval = the march): every stage input is
        # stored during the forward sweep (2 n_steps fields), nothing is recomputed
        plan.adjoint(u0, lam, 0, q.n_steps, q.n_steps)
        tall = _time(lambda: plan.adjoint(u0, lam, 0, q.n_steps, q.n_steps), sync)
        assert plan.poll() == 0
        out["adjoint_c5_" + dt] = {"fwd_s": tf, "adjoint_s": ta, "adjoint_over_fwd": ta / tf,
                                   "ckpt_every": inputs.C5_CKPT, "cache_assisted": True,
                                   "store_all": {"adjoint_s": tall, "adjoint_over_fwd": tall / tf,
                                                 "stored_bytes": 2 * q.n_steps * q.points * (4 if dt == "f32" else 8)}}
        progress("adjoint %s done" % dt)
        plan.close()
        del plan
    torch.cuda.empty_cache()
    # batched: 64 uneven solves in one plan, autotuned, the whole march replayed as one HIP graph
    probs = inputs.c4()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = kzk.Plan(probs, dtype="f32", stream=stream)
        u = plan.pack([pp.u0 for pp in probs])
        u0 = u.clone()
        tuned = plan.autotune(u, 3)
        plan.set_graph(True)
        plan.step(u, 0, 500)
        u.copy_(u0)
        tb = _time(lambda: plan.step(u, 0, 500), stream.synchronize)
        assert plan.poll() == 0
    pts = sum(pp.points for pp in probs)
    out["batched_c4_f32"] = {"solves": len(probs), "points": pts, "s_per_march": tb,
                             "value": pts * 500 / tb, "graph": True, "autotuned": plan.tuning()}
    progress("batched march done")
    plan.close()
    del plan, u, u0
    torch.cuda.empty_cache()
    out["paper_sets_f32"] = paper_sets()
    return out


def linear_march_error(state_fp64):
    """Relative l2 error of the FP32 2000-step 8192 x 4096 march with nl = 0
    (the workload's D(x) schedule and absorption) against its closed form:
    u0 = cos(k tau) exp(-y^2 / 2), u(x) = e^{-A k^2 x} Re[e^{i k tau} (1/sqrt(c))
    exp(-y^2 / (2 c))], c = 1 - i (int D dx) / k."""
    import math
    import numpy as np
    import torch
    from paper_2103_06080_amd import inputs, kzk
    p = inputs.c3()
    p.nl_node = np.zeros_like(p.nl_node)
    tau, y = p.tau(), p.y()
    k = 2 * math.pi * 3 / p.L_tau
    p.u0 = np.cos(k * tau)[None, :] * np.exp(-y ** 2 / 2)[:, None]
    plan = kzk.Plan(p, dtype="f32", state_fp64=state_fp64)
    u = plan.pack([p.u0])
    plan.step(u, 0, p.n_steps)
    assert plan.poll() == 0
    got = plan.unpack(u)[0]
    plan.close()
    del plan, u
    torch.cuda.empty_cache()
    c = 1 - 1j * float(p.h * p.D_step.sum()) / k
    ref = math.exp(-p.A * k * k * p.h * p.n_steps) * np.real(
        np.exp(1j * k * tau)[None, :] / np.sqrt(c) * np.exp(-y ** 2 / (2 * c))[:, None])
    return rel_l2(got, ref)


# Table 2 of the paper, CUDA FP32 column (Titan V), seconds for the whole run of
# each set on its own grid (N_theta = 7 * 2^k): context, not a target
PAPER_CUDA_FP32_S = {1: 0.5564, 2: 3.788, 3: 28.31, 4: 392.7}


def paper_sets():
    """The paper's workload (full b with transport by the random medium,
    regularised multiplier) on the grids of sets 1-4 (n_tau = N_theta = 7 2^k,
    n_y the power of two nearest N_rho) and on the power-of-two grids nearest
    them ("_pow2"), each run for its N_sigma steps in FP32 with per-kernel
    events on every 8th step.  value: grid-point-steps/s; paper_value: the
    same for the paper's CUDA FP32 time on its own grid (N_rho rows)."""
    import torch
    from paper_2103_06080_amd import inputs, kzk
    res = {}
    for k, pow2 in ((1, False), (2, False), (3, False), (4, False), (1, True), (2, True), (3, True), (4, True)):
        p = inputs.paper_set(k, pow2=pow2)
        plan = kzk.Plan(p, dtype="f32")
        u0 = plan.pack([p.u0])
        u = u0.clone()
        plan.step(u, 0, p.n_steps)
        assert plan.poll() == 0
        u.copy_(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(u, 0, p.n_steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        u.copy_(u0)
        plan.profile(True, every=PROFILE_EVERY)
        plan.step(u, 0, p.n_steps)
        prof = plan.profile_read()
        plan.profile(False)
        assert plan.poll() == 0
        ns, nrho, nth = inputs.PAPER_SETS[k]
        res["set%d%s" % (k, "_pow2" if pow2 else "")] = {"grid": [p.n_tau, p.n_y], "steps": p.n_steps, "s": t,
                            "value": p.points * p.n_steps / t,
                            "kernels_avg_us": {kk: round(1e3 * v[0] / v[1], 1) for kk, v in prof.items()},
                            "paper_grid": [nth, nrho], "paper_cuda_fp32_s": PAPER_CUDA_FP32_S[k],
                            "paper_value": nth * nrho * ns / PAPER_CUDA_FP32_S[k]}
        plan.close()
        del plan, u, u0
        torch.cuda.empty_cache()
        progress("paper set %d%s done" % (k, " (power-of-two grid)" if pow2 else ""))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0, help="seed of the synthetic field (c2, c3, c5)")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="no per-kernel events in the timed region")
    ap.add_argument("--y-threads", type=int, default=0, help="y-pass block size (0: plan default)")
    ap.add_argument("--tau-threads", type=int, default=0, help="tau-pass block size (0: plan default)")
    ap.add_argument("--tau-fft-radix", type=int, default=0, choices=[0, 8, 16],
                    help="radix schedule of the tau-transforms (0: plan default)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference for memory counters)")
    ap.add_argument("--march-steps", type=int, default=0, help="override the steps of one march (profiling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP64, adjoint and batched side measurements")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus %d requested); the multi-GPU "
              "decomposition is described in the design notes but not built" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2103_06080_amd import inputs, kzk

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    make = {"c3": inputs.c3, "c2": inputs.c2, "c5": inputs.c5}.get(args.config)
    prob = make(seed=args.seed) if make else inputs.c1()
    steps_per_march = min(args.march_steps or prob.n_steps, prob.n_steps)

    plan = kzk.Plan(prob, dtype=args.dtype, y_threads=args.y_threads or None, tau_threads=args.tau_threads or None,
                    tau_fft_radix=args.tau_fft_radix or None)
    u0 = plan.pack([prob.u0])
    u = torch.empty_like(u0)
    torch.cuda.synchronize()

    # every march (warm-up and timed) is the workload itself: steps 0 .. n-1
    # from the initial field, which stays resident in HBM (the copy into the
    # working field, 0.05 ms, is inside the timed region)
    def one_march():
        u.copy_(u0)
        plan.step(u, 0, steps_per_march)

    for _ in range(args.warmup):
        one_march()
    st = plan.poll()
    if st != 0:
        raise SystemExit("device status %d during warm-up" % st)

    if not args.no_profile:
        plan.profile(True, every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_march()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile_read() if not args.no_profile else {}
    plan.profile(False)
    st = plan.poll()
    if st != 0:
        raise SystemExit("device status %d in the timed region" % st)
    u_host = u.double().cpu().numpy().reshape(prob.n_y, prob.n_tau)
    assert np.isfinite(u_host).all()

    elapsed = t1 - t0
    progress("timed marches done (%.1f ms each)" % (1e3 * elapsed / args.steps))
    ms_per_step = 1e3 * elapsed / args.steps
    pts_steps = prob.points * steps_per_march * args.steps
    value = pts_steps / elapsed
    esz = 4 if args.dtype == "f32" else 8

    roofline = None
    kernels = {}
    if prof:
        for kind, (ms, cnt) in prof.items():
            kernels[kind] = {"launches": cnt, "avg_us": 1e3 * ms / cnt}
        dom = max((k for k in prof if k in ("tau_pass", "y_pass1", "y_pass2")), key=lambda k: prof[k][0])
        avg_s = prof[dom][0] / prof[dom][1] / 1e3
        nbytes, nflops = kernel_model(dom, prob.n_tau, prob.n_y, esz)
        gbs = nbytes / avg_s / 1e9
        tfl = nflops / avg_s / 1e12
        if gbs / HBM_PEAK_GBS >= tfl / ALU_PEAK_TFLOPS[args.dtype]:
            roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4)}
        else:
            roofline = {"bound": "alu", "achieved": round(tfl, 2), "peak": ALU_PEAK_TFLOPS[args.dtype],
                        "unit": "TFLOP/s", "frac": round(tfl / ALU_PEAK_TFLOPS[args.dtype], 4)}
        roofline["traffic"] = pmc_traffic(dom, args.config, args.dtype)
        roofline["kernel"] = dom
        roofline["avg_launch_us"] = round(avg_s * 1e6, 2)
        roofline["algorithmic_bytes_per_launch"] = nbytes
        roofline["algorithmic_flops_per_launch"] = nflops
        roofline["hbm_gbs_algorithmic"] = round(gbs, 1)
        roofline["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
        roofline["alu_frac_of_nonpacked_rate"] = round(tfl / NONPACKED_PEAK_TFLOPS, 4)
        # whole-step models: 11 array transfers per step (the minimal two-pass
        # model) and the 12 this build moves (it also writes the spectral state)
        step_bytes = esz * prob.points * steps_per_march * args.steps
        roofline["step_model_11_gbs"] = round(11 * step_bytes / elapsed / 1e9, 1)
        roofline["step_model_11_frac"] = round(11 * step_bytes / elapsed / 1e9 / HBM_PEAK_GBS, 4)
        roofline["step_model_12_gbs"] = round(12 * step_bytes / elapsed / 1e9, 1)
        # the same fractions against a measured device copy (1 GiB read + 1 GiB written)
        cp = measured_copy_gbs()
        roofline["measured_copy_gbs"] = round(cp, 1)
        roofline["hbm_frac_of_copy"] = round(gbs / cp, 4)
        roofline["step_model_11_frac_of_copy"] = round(11 * step_bytes / elapsed / 1e9 / cp, 4)

    tuning = plan.tuning()
    errors = {"full_march_sampled_rows": sampled_march_error(args.config, u_host, steps_per_march)
              if args.seed == 0 else None}
    plan.close()
    del plan, u, u0
    torch.cuda.empty_cache()

    extras = None
    if not args.no_extras and args.config == "c3" and not args.march_steps:
        extras = side_measurements(args, value, ms_per_step)

    cpu = None
    if not args.no_cpu_baseline:
        cpu, ref = cpu_baseline(prob)
        errors["first_steps"] = {dt: first_steps_error(prob, ref, dt) for dt in ("f32", "f64")}

    line = {
        "metric": "grid-point-steps/s",
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "%s: %s, %s" % (args.config, WORKLOADS[args.config], args.dtype), "seed": args.seed,
                   "n_tau": prob.n_tau, "n_y": prob.n_y, "march_steps": steps_per_march,
                   "x_range": [prob.x0, prob.x0 + prob.h * steps_per_march],
                   "tuning": tuning, "parallelism": "single GPU"},
        "rel_l2_vs_oracle": errors,
        "roofline": roofline,
        "kernels": kernels,
        "extras": extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
