#!/usr/bin/env python3
"""Benchmark: pair-interactions/s of RK4 shooting and time-to-match of the feedback iteration.

A step is one forward shoot through the C ABI (lm_shoot) of the headline workload: 65536
Fibonacci-sphere landmarks in 3-D, conical kernel sigma = 0.05, FP64, 100 RK4 steps on
[0, 1] from the template X with the workload's throughput momenta (a Jacobi estimate of the
first feedback momenta, so the kernel runs on realistic operands).  Every RK stage is one
pass of the O(N^2) pair sums with the stage bookkeeping fused in (equation "N-particle",
Algorithm 1 step 1).

value       = pair interactions of the timed shoots (steps * 4 * rk4_steps * N^2) / wall time
ms_per_step = wall time of one shoot.

Outside the timed loop, in this order, each only while the run's wall-clock budget
(--budget-s, counted from the start of the process) has room for it:
  - the dominant kernel's roofline (the RK stage, its time from HIP events recorded on the
    stream the library launches on, around every timed shoot);
  - the FP64 oracle timed on the host cores on a bounded sample (cpu_baseline);
  - time-to-match of the headline workload: Algorithm 1 from p = 0 until
    max|q(1) - Y| < 1e-6 (dense factor of K(X), shoots, solves), measured once, then once
    more with single-precision shoots until the residual is below 1e-5 and double after;
  - the single-precision form: the same shoot in FP32 (its stage time and roofline) and its
    error against the FP64 oracle's stored shoot, with the FP64 shoot's error beside it;
  - time-to-match of the 2-D curve (N = 4096, 200 RK4 steps, FP64, and FP32 switching to FP64)
    and of the circle -> ellipse (N = 64), and the FP32 curve shoot's error against the oracle;
  - the 256-problem batch (autotuned shape, batched shoots, batched Algorithm 1);
  - the differentiation workload (16384 sphere points, Gaussian sigma = 0.1, lambda = 100:
    energy gradient, L-BFGS, and the feedback iteration on the same problem).
A leg that does not fit is reported as skipped; the JSON line is always printed.

--mode match or iteration makes a step one whole match or one feedback iteration instead
(diagnostics; the headline is the shoot).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

T_START = time.time()

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")

# FP64 VALU issue slots charged per pair (an FMA is one slot, a quarter-rate transcendental
# four); fixed before any tuning and never changed, so a faster kernel shows up as a higher
# fraction of the roofline.
SLOTS_PER_PAIR = {(3, 0): 46, (2, 0): 41, (3, 1): 32, (2, 1): 27}
# The symmetric kernel evaluates each unordered pair once, N(N+1)/2 evaluations per launch,
# and charges the shared part once plus both particles' accumulations: S_pair + 2 dim slots.
# MI355X: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz = 3.93e13 FMA slots/s = 78.6 TFLOP/s
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9
PEAK_TFLOPS = 2.0 * PEAK_SLOTS / 1e12
# Single precision: the arithmetic of the FP64 charge plus v_exp_f32 (4 slots, with its
# range step 5) and, for the conon, v_rsq_f32 (4 slots, no Newton step at the FP32 bar),
# charged against MI355X's FP32 vector peak of 157.3 TFLOP/s (twice the FP64 lane rate).
SLOTS_PER_PAIR_F32 = {(3, 0): 28, (2, 0): 23, (3, 1): 22, (2, 1): 17}
PEAK_TFLOPS_F32 = 157.3

# HBM bytes per RK stage of the dominant kernel (the pair-sum launch and the launch that adds
# its partial sums) from rocprofv3 FETCH_SIZE and WRITE_SIZE runs,
# each scaled by the reading of a plain device copy of known size (fetch x2.000, write x1.000),
# recorded with the hash of the kernel sources they were taken on; a changed kernel reports
# null until the counters are taken again.
MEASURED_TRAFFIC = {
    "sphere3d_conon_f64": ("5cf04e6adfc45b06", 1.0439e9),
    "sphere3d_conon_f32": ("5cf04e6adfc45b06", 4.4403e8),
}

# Residual below which the headline's mixed-precision match moves from FP32 to FP64 shoots
F32_SWITCH = 1e-5

# Estimated seconds of each optional leg on MI355X (a leg runs only if the budget left
# covers it), refined in the run by what the headline shoot measured.
LEG_SECONDS = {"cpu_baseline": 20.0, "time_to_match": 40.0, "fp32": 15.0, "curve2d": 20.0,
               "batched": 90.0, "adjoint": 60.0}


def kernel_source_hash() -> str:
    import hashlib
    csrc = os.path.join(ROOT, "paper_1510_03816_amd", "csrc")
    data = b"".join(open(os.path.join(csrc, f), "rb").read()
                    for f in ("lm_kernels.hip", "lm_sym.hip", "lm_math.h"))
    return hashlib.sha256(data).hexdigest()[:16]


WORKLOADS = {
    # name: (generator kwargs, dtype); eps = kernel value at the tile-skipping radius
    "sphere3d_conon_f64": (dict(kind="sphere3d", n=65536, kernel=0, sigma=0.05, steps=100), 0),
    "sphere3d_conon_f32": (dict(kind="sphere3d", n=65536, kernel=0, sigma=0.05, steps=100), 1),
    "sphere3d_gauss_f64": (dict(kind="sphere3d", n=65536, kernel=1, sigma=0.05, steps=100), 0),
    "sphere3d_gauss_f64_cut": (dict(kind="sphere3d", n=65536, kernel=1, sigma=0.05, steps=100, eps=1e-16), 0),
    "sphere3d_conon_f64_cut": (dict(kind="sphere3d", n=65536, kernel=0, sigma=0.05, steps=100, eps=1e-16), 0),
    "sphere3d_conon_f32_cut": (dict(kind="sphere3d", n=65536, kernel=0, sigma=0.05, steps=100, eps=1e-10), 1),
    "curve2d_conon_f64": (dict(kind="curve2d", n=4096, kernel=0, sigma=0.1, steps=200), 0),
    "curve2d_conon_f32": (dict(kind="curve2d", n=4096, kernel=0, sigma=0.1, steps=200), 1),
    "circle_ellipse_f64": (dict(kind="circle_ellipse", n=64, kernel=0, sigma=0.5, steps=100), 0),
}


def make_problem(spec):
    import inputs
    if spec["kind"] == "sphere3d":
        return inputs.config_sphere3d(spec["n"], kernel=spec["kernel"], sigma=spec["sigma"], steps=spec["steps"])
    if spec["kind"] == "circle_ellipse":
        return inputs.config_circle_ellipse(spec["n"])
    return inputs.config_curve2d(spec["n"], kernel=spec["kernel"], sigma=spec["sigma"], steps=spec["steps"])


def cutoff_radius(spec) -> float:
    """Radius beyond which the kernel is below spec['eps'] (0 = every pair)."""
    eps = spec.get("eps")
    if not eps:
        return 0.0
    L = math.log(1.0 / eps)
    return spec["sigma"] * (L if spec["kernel"] == 0 else math.sqrt(L))


class Budget:
    """Wall-clock budget of the whole run, counted from the start of the process."""

    def __init__(self, seconds: float):
        self.seconds = seconds
        self.skipped = []

    def left(self) -> float:
        return self.seconds - (time.time() - T_START)

    def allows(self, leg: str, estimate: float) -> bool:
        if self.left() >= estimate:
            return True
        self.skipped.append(leg)
        log("budget: skipping %s (%.0f s left, needs about %.0f s)" % (leg, self.left(), estimate))
        return False


def cpu_baseline(pr, p, target_s: float):
    """The FP64 oracle on the host cores, on the same workload: one whole RK4 step of the
    shoot (four right-hand-side evaluations over all N^2 pairs) when that fits in about 2.5x
    the target time, else the rows of one RHS evaluation that fill the target time."""
    import numpy as np
    import oracle

    n = pr.n
    idx = np.linspace(0, n - 1, 64).astype(np.int64)
    t0 = time.perf_counter()
    oracle.rhs_rows(pr.X, p, idx, pr.kernel, pr.sigma)
    per_rhs = (time.perf_counter() - t0) * n / 64
    if 4 * per_rhs <= 2.5 * target_s:
        t0 = time.perf_counter()
        oracle.shoot(pr.X, p, pr.kernel, pr.sigma, 1, T=1.0 / pr.steps)
        dt = time.perf_counter() - t0
        return {"value": 4 * n * n / dt, "unit": "pair-interactions/s", "cores": oracle.num_threads(),
                "kind": "oracle",
                "sample": "one RK4 step (dt = 1/%d) of the %d-point shoot: 4 right-hand sides over all pairs, %.1f s"
                          % (pr.steps, n, dt)}
    rows = 64
    while True:
        idx = np.linspace(0, n - 1, rows).astype(np.int64)
        t0 = time.perf_counter()
        oracle.rhs_rows(pr.X, p, idx, pr.kernel, pr.sigma)
        dt = time.perf_counter() - t0
        if dt >= target_s or rows >= n:
            break
        rows = min(n, max(rows * 2, int(rows * target_s / max(dt, 1e-3) * 1.1)))
    return {"value": rows * n / dt, "unit": "pair-interactions/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d of the %d target rows of one RHS evaluation (all %d sources each), %.1f s"
                      % (rows, n, n, dt)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def stored_oracle(name: str, pr, p0):
    """The oracle's stored shoot of a workload (written by tests/golden/make_oracle_shoots.py),
    or None when it is absent or was made from other inputs."""
    import numpy as np
    path = os.path.join(GOLDEN, "oracle_shoot_%s.npz" % name)
    if not os.path.exists(path):
        return None
    z = np.load(path)
    idx = z["idx"]
    if int(z["n"]) != pr.n or not (np.allclose(z["X"], pr.X[:, idx], rtol=0, atol=1e-14)
                                   and np.allclose(z["p0"], p0[:, idx], rtol=0, atol=1e-14)):
        return None
    return z


def rel_err(got, want) -> float:
    import numpy as np
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def timed_shoots(lm, torch, prm, q0, p0, t1, steps, q1, p1, count):
    """Runs `count` shoots; returns (wall seconds, GPU milliseconds per shoot from HIP events
    recorded on the stream the library launches on)."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(count)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        st = lm.lm_shoot(prm, q0, p0, t1, steps, q1, p1)
        b.record()
        if st != 0:
            raise RuntimeError("lm_shoot: %s" % lm.STATUS_NAMES[st])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in evs]


def pair_roofline(lm, prm, n, dim, kernel, dtype, stage_ms, cutoff=0.0):
    """Roofline entry of one RK stage (pair-sum launch plus the launch adding its partials)."""
    plan = lm.lm_pair_plan(prm, n)
    kname = "%s,%d,%s,force" % ("double" if dtype == 0 else "float", dim, "conon" if kernel == 0 else "gauss")
    if dtype == 0:
        peak, table = PEAK_TFLOPS, SLOTS_PER_PAIR
    else:
        peak, table = PEAK_TFLOPS_F32, SLOTS_PER_PAIR_F32
    if plan["symmetric"]:
        slots = table[(dim, kernel)] + 2 * dim
        evals = n * (n + 1) // 2
        kname = "%s<%s> + lm_finish_kernel" % ("lm_sym_pair_wide_kernel" if plan["rows"] == 4 else "lm_sym_pair_kernel",
                                               kname)
    else:
        slots = table[(dim, kernel)]
        evals = n * n
        kname = "lm_pair_kernel<%s>%s" % (kname, " + lm_finish_kernel" if plan["partial_slots"] > 1 else "")
    achieved = evals * slots * 2.0 / (stage_ms * 1e-3) / 1e12
    if cutoff > 0.0:
        achieved = None          # with tile skipping fewer than N^2 pairs are evaluated
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": (achieved / peak) if achieved else None, "traffic": None,
            "kernel": kname, "plan": plan, "launch_ms": stage_ms, "pair_evaluations_per_launch": evals,
            "slots_per_evaluation": slots, "pairs_per_s_in_kernel": n * n / (stage_ms * 1e-3)}


def match_record(lm, st, info, seconds, tol, h):
    return {"seconds": seconds, "status": lm.STATUS_NAMES[st], "iters": info.iters, "resid_inf": info.resid_inf,
            "factor_ms": info.factor_ms, "shoot_ms": info.shoot_ms, "solve_ms": info.solve_ms,
            "cg_iters": info.cg_iters, "shoots": info.shoots, "tol": tol, "h": h, "paper_H_2H": 2 * info.H}


def fp32_leg(lm, torch, dev, pr, p_np, q64_gpu, p64_gpu):
    """The headline shoot in single precision: stage time, roofline, and its error against the
    oracle's stored FP64 shoot (and the FP64 GPU shoot's error beside it)."""
    prm = lm.make_params(pr.dim, pr.kernel, pr.sigma, dtype=lm.F32)
    q0 = torch.tensor(pr.X, device=dev, dtype=torch.float32)
    p0 = torch.tensor(p_np, device=dev, dtype=torch.float32)
    q1, p1 = torch.empty_like(q0), torch.empty_like(q0)
    timed_shoots(lm, torch, prm, q0, p0, 1.0, pr.steps, q1, p1, 1)                    # warm-up
    wall, ev = timed_shoots(lm, torch, prm, q0, p0, 1.0, pr.steps, q1, p1, 2)
    stage_ms = sum(ev) / (len(ev) * 4 * pr.steps)
    out = {"workload": "sphere3d_conon_f32", "shoot_ms": wall * 1e3 / 2,
           "pairs_per_s": 4 * pr.steps * pr.n ** 2 * 2 / wall,
           "roofline": pair_roofline(lm, prm, pr.n, pr.dim, pr.kernel, 1, stage_ms)}
    if MEASURED_TRAFFIC["sphere3d_conon_f32"][0] == kernel_source_hash():
        out["roofline"]["traffic"] = MEASURED_TRAFFIC["sphere3d_conon_f32"][1]
    q32, p32 = q1.double().cpu().numpy(), p1.double().cpu().numpy()
    q64, p64 = q64_gpu.cpu().numpy(), p64_gpu.cpu().numpy()
    out["err_vs_gpu_f64"] = {"q": rel_err(q32, q64), "p": rel_err(p32, p64)}
    z2 = stored_oracle("sphere3d_conon_2steps", pr, p_np)
    if z2 is not None:
        # the first two RK4 steps of the same shoot, FP32 and FP64, against the oracle's
        idx = z2["idx"]
        errs = {}
        for name, dt_ in [("f32", torch.float32), ("f64", torch.float64)]:
            prm2 = lm.make_params(pr.dim, pr.kernel, pr.sigma, dtype=lm.F32 if dt_ == torch.float32 else lm.F64)
            a = torch.tensor(pr.X, device=dev, dtype=dt_)
            b = torch.tensor(p_np, device=dev, dtype=dt_)
            qa, pa = torch.empty_like(a), torch.empty_like(a)
            lm.lm_shoot(prm2, a, b, float(z2["T"]), int(z2["steps"]), qa, pa)
            qh, ph = qa.double().cpu().numpy()[:, idx], pa.double().cpu().numpy()[:, idx]
            errs[name] = {"q": rel_err(qh, z2["q1"]), "p": rel_err(ph, z2["p1"])}
        out["err_vs_oracle_2steps"] = dict(errs, rows=int(len(idx)), bars={"f32": 1e-4, "f64": 1e-10})
    z = stored_oracle("sphere3d_conon_100steps", pr, p_np)
    if z is not None:
        idx = z["idx"]
        out["err_vs_oracle"] = {"q": rel_err(q32[:, idx], z["q1"]), "p": rel_err(p32[:, idx], z["p1"]),
                                "rows": int(len(idx)), "bar": 1e-4}
        out["f64_err_vs_oracle"] = {"q": rel_err(q64[:, idx], z["q1"]), "p": rel_err(p64[:, idx], z["p1"]),
                                    "rows": int(len(idx)), "bar": 1e-10}
    log("fp32 shoot: %.1f ms, stage %.3f ms, err vs FP64 gpu q %.2e p %.2e%s" % (
        out["shoot_ms"], stage_ms, out["err_vs_gpu_f64"]["q"], out["err_vs_gpu_f64"]["p"],
        (", vs oracle q %.2e p %.2e" % (out["err_vs_oracle"]["q"], out["err_vs_oracle"]["p"]))
        if "err_vs_oracle" in out else ""))
    return out


def curve2d_leg(lm, torch, dev, h, tol, setup, run_match):
    """2-D curve (N = 4096, 200 RK4 steps) and circle -> ellipse (N = 64) time-to-match, and the
    curve's FP32 and FP64 shoots against the oracle's stored shoot."""
    out = {}
    for mname, sw in [("curve2d_conon_f64", 0.0), ("curve2d_conon_f32", 1e-4), ("circle_ellipse_f64", 0.0)]:
        mpr, mdtype, mrc, mprm, MX, MY = setup(mname)
        run_match(mprm, mpr, MX, MY, sw)                     # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, minfo, _ = run_match(mprm, mpr, MX, MY, sw)
        torch.cuda.synchronize()
        rec = match_record(lm, st, minfo, time.perf_counter() - t1, tol, h)
        rec.update(workload=mname, n=mpr.n, f32_switch=sw)
        out[mname] = rec
        log("time to match %s: %.3f s, %d iterations, resid %.2e" % (mname, rec["seconds"], minfo.iters,
                                                                      minfo.resid_inf))
    pr = make_problem(WORKLOADS["curve2d_conon_f64"][0])
    p_np = pr.p_bench()
    z = stored_oracle("curve2d_conon_200steps", pr, p_np)
    if z is not None:
        idx = z["idx"]
        errs = {}
        for name, dt_ in [("f64", torch.float64), ("f32", torch.float32)]:
            prm = lm.make_params(2, pr.kernel, pr.sigma, dtype=lm.F64 if dt_ == torch.float64 else lm.F32)
            q0 = torch.tensor(pr.X, device=dev, dtype=dt_)
            p0 = torch.tensor(p_np, device=dev, dtype=dt_)
            q1, p1 = torch.empty_like(q0), torch.empty_like(q0)
            lm.lm_shoot(prm, q0, p0, 1.0, pr.steps, q1, p1)
            q, p = q1.double().cpu().numpy()[:, idx], p1.double().cpu().numpy()[:, idx]
            errs[name] = {"q": rel_err(q, z["q1"]), "p": rel_err(p, z["p1"])}
        out["shoot_err_vs_oracle"] = dict(errs, rows=int(len(idx)), bars={"f64": 1e-10, "f32": 1e-4})
        log("curve2d shoot vs oracle: f64 q %.2e p %.2e, f32 q %.2e p %.2e" % (
            errs["f64"]["q"], errs["f64"]["p"], errs["f32"]["q"], errs["f32"]["p"]))
    return out


def batched_leg(lm, torch, dev, h: float, tol: float):
    """The 256-problem batch: autotuned shape, shoot throughput, time-to-match."""
    import numpy as np
    import inputs

    sizes, offs, X, Y = inputs.config_batched()
    steps = 100
    pairs = float((sizes.astype(np.float64) ** 2).sum())
    p = np.concatenate([inputs.bench_momentum(X[:, offs[b]:offs[b + 1]], Y[:, offs[b]:offs[b + 1]],
                                              inputs.curve_kernel_mass(int(sizes[b]), 2 * math.pi, 0.1, 0))
                        for b in range(len(sizes))], axis=1)
    Xd, Yd = torch.tensor(X, device=dev), torch.tensor(Y, device=dev)
    out = {"workload": "batched256_curve2d_conon", "problems": int(len(sizes)), "n_total": int(offs[-1]),
           "n_min": int(sizes.min()), "n_max": int(sizes.max()), "sum_n2": pairs, "rk4_steps": steps,
           "sigma": 0.1}
    tunings = {}
    for name, dtype, tdt in [("f32", lm.F32, torch.float32), ("f64", lm.F64, torch.float64)]:
        prm = lm.make_params(2, lm.CONON, 0.1, dtype=dtype)
        q0, p0 = Xd.to(tdt), torch.tensor(p, dtype=tdt, device=dev)
        t = lm.lm_batch_autotune(prm, offs, q0, p0)
        tunings[name] = t
        q1, p1 = torch.empty_like(q0), torch.empty_like(q0)
        lm.lm_shoot_batched(prm, offs, q0, p0, 1.0, steps, q1, p1, tuning=t)       # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lm.lm_shoot_batched(prm, offs, q0, p0, 1.0, steps, q1, p1, tuning=t)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["shoot_" + name] = {"ms": dt * 1e3, "pairs_per_s": pairs * 4 * steps / dt, "tuning": t.as_dict()}
        # the same shoot with every kernel launched directly and with 20 RK4 steps per replayed
        # hipGraph, whatever the tuner chose
        cmp_ = {}
        for gs in (0, 20):
            tg = lm.lm_batch_tuning.from_buffer_copy(t)
            tg.graph_steps = gs
            lm.lm_shoot_batched(prm, offs, q0, p0, 1.0, steps, q1, p1, tuning=tg)       # capture / warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lm.lm_shoot_batched(prm, offs, q0, p0, 1.0, steps, q1, p1, tuning=tg)
            torch.cuda.synchronize()
            cmp_["graph_steps_%d_ms" % gs] = (time.perf_counter() - t0) * 1e3
        out["shoot_" + name]["launch_comparison"] = cmp_
        log("batched shoot %s: %.1f ms, %.3e pairs/s (tuning %s)" % (name, dt * 1e3, pairs * 4 * steps / dt,
                                                                    t.as_dict()))
    for name, dtype, sw in [("f32_then_f64", lm.F32, 1e-4), ("f64", lm.F64, 0.0)]:
        prm = lm.make_params(2, lm.CONON, 0.1, dtype=dtype)
        pg = torch.zeros_like(Xd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, infos, stats = lm.lm_feedback_match_batched(prm, offs, Xd, Yd, pg, h=h, tol=tol, steps=steps,
                                                        max_iter=200, tuning=tunings["f32" if dtype == lm.F32
                                                                                     else "f64"],
                                                        f32_switch=sw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        its = [i.iters for i in infos]
        out["time_to_match_" + name] = {
            "seconds": dt, "status": lm.STATUS_NAMES[st], "converged": sum(1 for s in stats if s == 0),
            "iters_max": max(its), "iters_mean": sum(its) / len(its),
            "shoots_max": max(i.shoots for i in infos),
            "resid_max": max(i.resid_inf for i in infos), "shoot_ms": infos[0].shoot_ms,
            "solve_ms": infos[0].solve_ms, "factor_ms": infos[0].factor_ms, "tol": tol, "h": h,
            "f32_switch": sw}
        log("batched time to match (%s): %.2f s, %s, iterations max %d" % (name, dt, lm.STATUS_NAMES[st], max(its)))
    return out


def adjoint_leg(lm, torch, dev, full: bool):
    """Gradient-based matching on the differentiation workload (16384 Fibonacci-sphere points,
    Gaussian sigma = 0.1, lambda = 100, 100 RK4 steps, checkpoints every 10 steps) beside the
    feedback iteration on the same problem."""
    import inputs

    pr = inputs.config_adjoint3d()
    lam, ck = pr.extra["lam"], pr.extra["ckpt_every"]
    prm = lm.make_params(3, lm.GAUSS, pr.sigma)
    X, Y = torch.tensor(pr.X, device=dev), torch.tensor(pr.Y, device=dev)
    out = {"workload": "adjoint3d_gauss_f64", "n": pr.n, "sigma": pr.sigma, "lam": lam, "rk4_steps": pr.steps,
           "ckpt_every": ck}
    p0, g = torch.zeros_like(X), torch.empty_like(X)
    lm.lm_energy_grad(prm, X, Y, p0, lam, pr.steps, g, ckpt_every=ck)           # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lm.lm_energy_grad(prm, X, Y, p0, lam, pr.steps, g, ckpt_every=ck)
    torch.cuda.synchronize()
    out["energy_grad_s"] = time.perf_counter() - t0
    runs = [("lbfgs_energy", 1.0, 1e-6, 0.0)]
    if full:
        runs.append(("lbfgs_data_term_to_1e-6", 0.0, 0.0, 1e-6))
    for name, reg, gtol, mtol in runs:
        p0 = torch.zeros_like(X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, info = lm.lm_lbfgs_match(prm, X, Y, p0, lam=lam, steps=pr.steps, reg=reg, gtol=gtol, match_tol=mtol,
                                     max_iter=300, history=16, ckpt_every=ck)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"seconds": dt, "status": lm.STATUS_NAMES[st], "iters": info.iters, "evals": info.evals,
                     "E": info.E, "gnorm_inf": info.gnorm_inf, "resid_inf": info.resid_inf, "reg": reg,
                     "gtol": gtol, "match_tol": mtol}
        log("adjoint %s: %s %.1f s, %d iterations, %d evaluations, endpoint error %.2e" % (
            name, lm.STATUS_NAMES[st], dt, info.iters, info.evals, info.resid_inf))
    p0 = torch.zeros_like(X)
    t0 = time.perf_counter()
    st, info, _ = lm.lm_feedback_match(prm, X, Y, p0, h=0.8, tol=1e-6, steps=pr.steps, max_iter=30,
                                       solver=lm.SOLVE_DENSE)
    out["feedback_dense"] = {"seconds": time.perf_counter() - t0, "status": lm.STATUS_NAMES[st],
                             "message": lm.last_error() if st != 0 else ""}
    log("adjoint workload, feedback iteration: %s" % lm.STATUS_NAMES[st])
    return out


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed steps (forward shoots)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed steps before")
    ap.add_argument("--workload", default="sphere3d_conon_f64", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="shoot", choices=["shoot", "match", "iteration"],
                    help="a step is one forward shoot from the workload's benchmark momenta (default), one "
                         "whole match, or one feedback iteration")
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="wall-clock budget of the whole run from process start; the legs after the timed "
                         "steps are skipped when it has no room for them")
    ap.add_argument("--h", type=float, default=0.8, help="search length of Algorithm 1")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--solver", type=int, default=0, help="0 auto (dense if it fits), 1 CG, 2 dense")
    ap.add_argument("--cg-max-iter", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-match", action="store_true", help="skip the headline workload's time-to-match")
    ap.add_argument("--no-fp32", action="store_true", help="skip the single-precision shoot")
    ap.add_argument("--no-curve2d", action="store_true", help="skip the 2-D curve and circle workloads")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-problem batch measurements")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the gradient-matching measurements")
    ap.add_argument("--adjoint-full", action="store_true",
                    help="also time L-BFGS on the data term alone to max|q(1) - Y| < 1e-6 (about 90 s)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the gradient-matching measurements (a diagnostic line, not the benchmark)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the 256-problem batch measurements (a diagnostic line, not the benchmark)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference for HBM byte counters)")
    return ap.parse_args(argv)


def main():
    args = parse_args()

    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; the pair sums would shard by target rows with one "
              "all-gather of (q, p) per RK stage, which the library does not implement. Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1510_03816_amd as lm

    budget = Budget(args.budget_s)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * 131072, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read, %d MiB written" % (args.calibrate_copy, args.calibrate_copy))
        del src, dst

    if args.batched_only:
        print(json.dumps({"batched": batched_leg(lm, torch, dev, args.h, args.tol)}), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_leg(lm, torch, dev, args.adjoint_full)}), flush=True)
        return

    def setup(name):
        spec, dtype = WORKLOADS[name]
        pr = make_problem(spec)
        rc = cutoff_radius(spec)
        prm = lm.make_params(pr.dim, pr.kernel, pr.sigma, dtype=dtype, cutoff=rc)
        X = torch.tensor(pr.X, device=dev)
        Y = torch.tensor(pr.Y, device=dev)
        return pr, dtype, rc, prm, X, Y

    def run_match(prm, pr, X, Y, f32_switch=0.0):
        p = torch.zeros_like(X)
        return lm.lm_feedback_match(prm, X, Y, p, h=args.h, tol=args.tol, steps=pr.steps,
                                    max_iter=args.max_iter, cg_max_iter=args.cg_max_iter, solver=args.solver,
                                    f32_switch=f32_switch)

    pr, dtype, rc, prm, X, Y = setup(args.workload)
    n, dim = pr.n, pr.dim
    pairs_per_shoot = 4 * pr.steps * n * n
    log("workload %s: N=%d dim=%d kernel=%s sigma=%g rk4_steps=%d dtype=%s cutoff=%g mode=%s" % (
        args.workload, n, dim, "conon" if pr.kernel == 0 else "gauss", pr.sigma, pr.steps,
        "f64" if dtype == 0 else "f32", rc, args.mode))

    sdt = torch.float64 if dtype == 0 else torch.float32
    p_np = pr.p_bench()
    q_sh = X.to(sdt)
    p_sh = torch.tensor(p_np, device=dev, dtype=sdt)
    q1_sh, p1_sh = torch.empty_like(q_sh), torch.empty_like(q_sh)
    p_iter = torch.zeros_like(X)
    records = []
    gpu_ms = {"shoot": 0.0, "solve": 0.0, "factor": 0.0}

    if args.mode == "shoot":
        if args.warmup > 0:
            timed_shoots(lm, torch, prm, q_sh, p_sh, 1.0, pr.steps, q1_sh, p1_sh, args.warmup)
        elapsed, ev_ms = timed_shoots(lm, torch, prm, q_sh, p_sh, 1.0, pr.steps, q1_sh, p1_sh, args.steps)
        shoots = args.steps
        gpu_ms["shoot"] = sum(ev_ms)
        records = [{"shoot_ms_gpu": t} for t in ev_ms]
        log("timed %d shoots: %.1f ms each (wall), GPU %.1f .. %.1f ms" % (
            shoots, elapsed * 1e3 / shoots, min(ev_ms), max(ev_ms)))
    else:
        def step():
            if args.mode == "match":
                st, info, _ = run_match(prm, pr, X, Y)
                rec = {"status": lm.STATUS_NAMES[st], "iters": info.iters, "resid_inf": info.resid_inf,
                       "factor_ms": info.factor_ms, "shoot_ms": info.shoot_ms, "solve_ms": info.solve_ms}
                return info.shoots, info.shoot_ms, info.solve_ms, info.factor_ms, rec
            st, info = lm.lm_feedback_step(prm, X, Y, p_iter, h=args.h, tol=args.tol, steps=pr.steps,
                                           cg_max_iter=args.cg_max_iter, solver=lm.SOLVE_CG)
            rec = {"status": lm.STATUS_NAMES[st], "resid_inf": info.resid_inf, "cg_iters": info.cg_iters,
                   "shoot_ms": info.shoot_ms, "solve_ms": info.solve_ms}
            return 1, info.shoot_ms, info.solve_ms, 0.0, rec

        for _ in range(args.warmup):
            step()
        p_iter.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        shoots = 0
        for _ in range(args.steps):
            s, a, b, c, rec = step()
            shoots += s
            gpu_ms["shoot"] += a
            gpu_ms["solve"] += b
            gpu_ms["factor"] += c
            records.append(rec)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0

    value = pairs_per_shoot * shoots / elapsed
    stage_ms = gpu_ms["shoot"] / (shoots * 4 * pr.steps)
    roofline = pair_roofline(lm, prm, n, dim, pr.kernel, dtype, stage_ms, rc)
    if args.workload in MEASURED_TRAFFIC and MEASURED_TRAFFIC[args.workload][0] == kernel_source_hash():
        roofline["traffic"] = MEASURED_TRAFFIC[args.workload][1]
    roofline["traffic_unit"] = "HBM bytes per RK stage (pair-sum and finish launches)"
    roofline["timing"] = "HIP events on the library's stream around every timed shoot / (4 x RK4 steps)"
    shoot_s = elapsed / max(shoots, 1)
    log("roofline: %.3f ms per stage, %.1f TFLOP/s, frac %.3f" % (
        stage_ms, roofline["achieved"] or 0.0, roofline["frac"] or 0.0))

    legs = {}

    def leg(name, fn, estimate):
        if not budget.allows(name, estimate):
            legs[name] = {"skipped": "wall-clock budget"}
            return None
        t = time.time()
        try:
            r = fn()
        except Exception as e:              # report the leg's failure and keep the line
            log("%s failed: %r" % (name, e))
            r = {"error": repr(e)}
        log("%s leg: %.1f s" % (name, time.time() - t))
        return r

    cpu = None
    if not args.no_cpu_baseline:
        cpu = leg("cpu_baseline", lambda: cpu_baseline(pr, p_np, args.cpu_seconds), args.cpu_seconds * 2.5 + 5)

    ttm = None
    if not args.no_match and args.mode == "shoot" and rc == 0.0:
        def ttm_fn():
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, info, _ = run_match(prm, pr, X, Y)
            torch.cuda.synchronize()
            r = match_record(lm, st, info, time.perf_counter() - t1, args.tol, args.h)
            r.update(workload=args.workload)
            log("time to match %s: %.2f s, %d iterations, resid %.2e" % (args.workload, r["seconds"], info.iters,
                                                                          info.resid_inf))
            return r
        ttm = leg("time_to_match", ttm_fn, max(LEG_SECONDS["time_to_match"], 22 * shoot_s))

        def ttm_mixed_fn():
            # the same match with single-precision shoots until the residual falls below 1e-5,
            # double-precision shoots after (momenta, residuals and K-solves always in double).
            # The FP32 shoot's endpoint error on this workload is about 1e-6 against the oracle,
            # so residuals down to 1e-5 are resolved: the residual history is the FP64 one to two
            # digits at every switch from 1e-4 to 1e-5, and single precision's floor is 3e-6.
            prm32 = lm.make_params(pr.dim, pr.kernel, pr.sigma, dtype=lm.F32)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, info, _ = run_match(prm32, pr, X, Y, F32_SWITCH)
            torch.cuda.synchronize()
            r = match_record(lm, st, info, time.perf_counter() - t1, args.tol, args.h)
            r.update(workload=args.workload, f32_switch=F32_SWITCH)
            log("time to match %s, FP32 shoots switching to FP64 below %g: %.2f s, %d iterations, resid %.2e" % (
                args.workload, F32_SWITCH, r["seconds"], info.iters, info.resid_inf))
            return r
        if args.workload == "sphere3d_conon_f64" and isinstance(ttm, dict) and "seconds" in ttm:
            ttm["f32_switch_run"] = leg("time_to_match_f32_switch", ttm_mixed_fn, 0.8 * ttm["seconds"] + 5)
    elif args.mode == "match":
        ttm = dict(records[-1], workload=args.workload, seconds=elapsed / args.steps, tol=args.tol, h=args.h)

    fp32 = None
    if not args.no_fp32 and args.workload == "sphere3d_conon_f64" and args.mode == "shoot":
        fp32 = leg("fp32", lambda: fp32_leg(lm, torch, dev, pr, p_np, q1_sh, p1_sh),
                   max(LEG_SECONDS["fp32"], 4 * shoot_s))

    curves = None
    if not args.no_curve2d:
        curves = leg("curve2d", lambda: curve2d_leg(lm, torch, dev, args.h, args.tol, setup, run_match),
                     LEG_SECONDS["curve2d"])
    batched = None if args.no_batched else leg("batched", lambda: batched_leg(lm, torch, dev, args.h, args.tol),
                                               LEG_SECONDS["batched"])
    adjoint = None if args.no_adjoint else leg("adjoint", lambda: adjoint_leg(lm, torch, dev, args.adjoint_full),
                                               LEG_SECONDS["adjoint"] + (90.0 if args.adjoint_full else 0.0))

    out = {
        "metric": "pair-interactions/s (RK4 shooting) + time-to-match at endpoint err 1e-6",
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dtype == 0 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "dim": dim,
                   "kernel": "conon" if pr.kernel == 0 else "gauss", "sigma": pr.sigma,
                   "rk4_steps": pr.steps, "h": args.h, "tol": args.tol, "cutoff": rc,
                   "step": {"shoot": "one forward shoot of the RK4 steps from X with the benchmark momenta",
                            "match": "one whole feedback match from p = 0 to max|q(1) - Y| < tol",
                            "iteration": "one feedback iteration (CG K-solve)"}[args.mode]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_match": ttm,
        "fp32": fp32,
        "curve2d": curves,
        "batched": batched,
        "adjoint": adjoint,
        "legs_skipped": budget.skipped,
        "wall_s": time.time() - T_START,
        "shoots": shoots,
        "gpu_ms": gpu_ms,
        "records": records,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
