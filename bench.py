#!/usr/bin/env python3
"""Benchmark: pair-interactions/s of RK4 shooting and time-to-match of the feedback iteration.

A step is one whole match through the C ABI (lm_feedback_match): Algorithm 1 from p = 0 (the
paper's initial guess) until max|q(1) - Y| < 1e-6 -- the factorisation of K(X) once, then
per iteration an RK4 shoot of the N-particle system (every stage one pass of the O(N^2)
pair sums, the stage bookkeeping fused in), the max-norm residual and the momentum update
p <- p + h K(X)^{-1} e.  Every row of the hot path runs inside the timed region.

value       = shooting pair interactions of the step (shoots * 4 * rk4_steps * N^2) / its
              wall time (factorisation, solves and residuals count against it)
ms_per_step = time to match.
Beside them: the dominant kernel's roofline (its average launch time measured live with HIP
events on the stream it runs on, inside the library), time-to-match on the 2-D curve (N =
4096) and circle-to-ellipse (N = 64) workloads, and the FP64 oracle timed on the host cores
on a bounded sample.

Also reported (not part of value): the 256-problem batch (2-D curves, N_b log-uniform in
[32, 4096], conical sigma = 0.1, 100 RK4 steps) -- autotuned launch shape, batched shoot
pair-interactions/s in FP32 and FP64, and batched time-to-match at 1e-6 (FP32 shoots
switching to FP64 at residual 1e-4, and FP64 throughout).

And the differentiation workload (16384 sphere points, Gaussian sigma = 0.1, lambda = 100):
one energy-and-gradient evaluation, L-BFGS on the energy, and the feedback iteration on the
same problem (its Gaussian kernel matrix is numerically singular there).

Default workload: 65536 Fibonacci-sphere landmarks in 3-D, conical kernel sigma = 0.05,
100 RK4 steps on [0, 1], FP64, h = 0.8; the target is the template moved by a seeded smooth
field.  --mode iteration times single feedback iterations (lm_feedback_step, CG K-solve)
instead, for workloads whose kernel matrix is singular (the Gaussian at these widths).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# FP64 VALU issue slots charged per pair (an FMA is one slot, a quarter-rate transcendental
# four); fixed before any tuning and never changed, so a faster kernel shows up as a higher
# fraction of the roofline.
SLOTS_PER_PAIR = {(3, 0): 46, (2, 0): 41, (3, 1): 32, (2, 1): 27}
# The symmetric kernel evaluates each unordered pair once, N(N+1)/2 evaluations per launch,
# and charges the shared part once plus both particles' accumulations: S_pair + 2 dim slots.
# MI355X: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz = 3.93e13 FMA slots/s = 78.6 TFLOP/s
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9
PEAK_TFLOPS = 2.0 * PEAK_SLOTS / 1e12

# HBM bytes per RK stage of the dominant kernel (the pair-sum launch and the launch that adds
# its partial sums) from rocprofv3 FETCH_SIZE and WRITE_SIZE runs,
# each scaled by the reading of a plain device copy of known size (fetch x2.000, write x1.000),
# recorded with the hash of the kernel sources they were taken on; a changed kernel reports
# null until the counters are taken again.
MEASURED_TRAFFIC = {
    "sphere3d_conon_f64": ("f6c3a5cf97caf2d9", 1.0588e9),
}


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


def cpu_baseline(pr, target_s: float):
    """The FP64 oracle on the host cores: rows of one RHS evaluation of the same workload."""
    import numpy as np
    import oracle

    n = pr.n
    p = pr.p_bench()
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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1, help="timed steps (whole matches)")
    ap.add_argument("--warmup", type=int, default=1, help="untimed steps before")
    ap.add_argument("--workload", default="sphere3d_conon_f64", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="match", choices=["match", "iteration", "shoot"],
                    help="a step is one whole match, one feedback iteration, or one forward shoot from the "
                         "workload's benchmark momenta")
    ap.add_argument("--h", type=float, default=0.8, help="search length of Algorithm 1")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--solver", type=int, default=0, help="0 auto (dense if it fits), 1 CG, 2 dense")
    ap.add_argument("--cg-max-iter", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--match", default="curve2d_conon_f64,circle_ellipse_f64",
                    help="comma-separated workloads whose time-to-match is also reported (outside value), "
                         "or none")
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
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; the pair sums would shard by target rows with one "
              "all-gather of (q, p) per RK stage, which is not built here. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1510_03816_amd as lm

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

    def run_match(prm, pr, X, Y):
        p = torch.zeros_like(X)
        return lm.lm_feedback_match(prm, X, Y, p, h=args.h, tol=args.tol, steps=pr.steps,
                                    max_iter=args.max_iter, cg_max_iter=args.cg_max_iter, solver=args.solver)

    pr, dtype, rc, prm, X, Y = setup(args.workload)
    n, dim = pr.n, pr.dim
    pairs_per_shoot = 4 * pr.steps * n * n
    log("workload %s: N=%d dim=%d kernel=%s sigma=%g rk4_steps=%d dtype=%s cutoff=%g mode=%s" % (
        args.workload, n, dim, "conon" if pr.kernel == 0 else "gauss", pr.sigma, pr.steps,
        "f64" if dtype == 0 else "f32", rc, args.mode))

    p_iter = torch.zeros_like(X)
    if args.mode == "shoot":
        sdt = torch.float64 if dtype == 0 else torch.float32
        q_sh = X.to(sdt)
        p_sh = torch.tensor(pr.p_bench(), device=dev, dtype=sdt)
        q1_sh, p1_sh = torch.empty_like(q_sh), torch.empty_like(q_sh)

    def step():
        """Returns (shoots, shoot_ms, solve_ms, factor_ms, record)."""
        if args.mode == "shoot":
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = lm.lm_shoot(prm, q_sh, p_sh, 1.0, pr.steps, q1_sh, p1_sh)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1e3
            log("shoot: %s %.1f ms" % (lm.STATUS_NAMES[st], ms))
            return 1, ms, 0.0, 0.0, {"status": lm.STATUS_NAMES[st], "shoot_ms": ms}
        if args.mode == "match":
            st, info, hist = run_match(prm, pr, X, Y)
            rec = {"status": lm.STATUS_NAMES[st], "iters": info.iters, "resid_inf": info.resid_inf,
                   "cg_iters": info.cg_iters, "factor_ms": info.factor_ms, "shoot_ms": info.shoot_ms,
                   "solve_ms": info.solve_ms, "paper_H_2H": 2 * info.H}
            log("match: %s %d iterations, resid %.3e, factor %.0f ms, shoots %.0f ms, solves %.0f ms" % (
                rec["status"], info.iters, info.resid_inf, info.factor_ms, info.shoot_ms, info.solve_ms))
            return info.iters + 1, info.shoot_ms, info.solve_ms, info.factor_ms, rec
        st, info = lm.lm_feedback_step(prm, X, Y, p_iter, h=args.h, tol=args.tol, steps=pr.steps,
                                       cg_max_iter=args.cg_max_iter, solver=lm.SOLVE_CG)
        rec = {"status": lm.STATUS_NAMES[st], "resid_inf": info.resid_inf, "cg_iters": info.cg_iters,
               "shoot_ms": info.shoot_ms, "solve_ms": info.solve_ms}
        log("iteration: %s resid %.3e shoot %.0f ms solve %.0f ms (%d CG)" % (
            rec["status"], info.resid_inf, info.shoot_ms, info.solve_ms, info.cg_iters))
        return 1, info.shoot_ms, info.solve_ms, 0.0, rec

    for _ in range(args.warmup):
        step()
    p_iter.zero_()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    shoots = 0
    shoot_ms = solve_ms = factor_ms = 0.0
    records = []
    for _ in range(args.steps):
        s, a, b, c, rec = step()
        shoots += s
        shoot_ms += a
        solve_ms += b
        factor_ms += c
        records.append(rec)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    value = pairs_per_shoot * shoots / elapsed
    # dominant kernel: the pair-sum kernel, one launch per RK stage
    launch_ms = shoot_ms / (shoots * 4 * pr.steps)
    plan = lm.lm_pair_plan(prm, n)
    kname = "%s,%d,%s,force" % ("double" if dtype == 0 else "float", dim, "conon" if pr.kernel == 0 else "gauss")
    if plan["symmetric"]:
        slots = SLOTS_PER_PAIR[(dim, pr.kernel)] + 2 * dim
        evals = n * (n + 1) // 2
        kname = "%s<%s> + lm_finish_kernel" % ("lm_sym_pair_wide_kernel" if plan["rows"] == 4 else "lm_sym_pair_kernel",
                                               kname)
    else:
        slots = SLOTS_PER_PAIR[(dim, pr.kernel)]
        evals = n * n
        kname = "lm_pair_kernel<%s>%s" % (kname, " + lm_finish_kernel" if plan["partial_slots"] > 1 else "")
    achieved = evals * slots * 2.0 / (launch_ms * 1e-3) / 1e12
    if rc > 0.0:
        # with tile skipping the pairs evaluated are fewer than N^2: not a roofline figure
        achieved = None
    traffic = None
    if args.workload in MEASURED_TRAFFIC and MEASURED_TRAFFIC[args.workload][0] == kernel_source_hash():
        traffic = MEASURED_TRAFFIC[args.workload][1]
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": (achieved / PEAK_TFLOPS) if achieved else None, "traffic": traffic,
                "traffic_unit": "HBM bytes per RK stage (pair-sum and finish launches)",
                "kernel": kname, "plan": plan,
                "launch_ms": launch_ms, "pair_evaluations_per_launch": evals, "slots_per_evaluation": slots,
                "pairs_per_s_in_kernel": n * n / (launch_ms * 1e-3)}

    ttm = None
    if args.mode == "match":
        ttm = dict(records[-1], workload=args.workload, seconds=elapsed / args.steps, tol=args.tol, h=args.h)

    extra_matches = {}
    for mname in ([] if args.match == "none" else args.match.split(",")):
        if mname == args.workload:
            continue
        mpr, mdtype, mrc, mprm, MX, MY = setup(mname)
        run_match(mprm, mpr, MX, MY)                         # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, minfo, hist = run_match(mprm, mpr, MX, MY)
        torch.cuda.synchronize()
        extra_matches[mname] = {
            "workload": mname, "n": mpr.n, "seconds": time.perf_counter() - t1, "status": lm.STATUS_NAMES[st],
            "iters": minfo.iters, "resid_inf": minfo.resid_inf, "factor_ms": minfo.factor_ms,
            "shoot_ms": minfo.shoot_ms, "solve_ms": minfo.solve_ms, "cg_iters": minfo.cg_iters,
            "tol": args.tol, "h": args.h, "paper_H_2H": 2 * minfo.H}
        log("time to match %s: %.3f s, %d iterations, resid %.2e" % (
            mname, extra_matches[mname]["seconds"], minfo.iters, minfo.resid_inf))
    ttm2 = extra_matches.get("curve2d_conon_f64")
    ttm3 = extra_matches.get("circle_ellipse_f64")

    batched = None if args.no_batched else batched_leg(lm, torch, dev, args.h, args.tol)
    adjoint = None if args.no_adjoint else adjoint_leg(lm, torch, dev, args.adjoint_full)

    cpu = None if args.no_cpu_baseline else cpu_baseline(pr, args.cpu_seconds)

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
                   "step": {"match": "one whole feedback match from p = 0 to max|q(1) - Y| < tol",
                            "iteration": "one feedback iteration (CG K-solve)",
                            "shoot": "one forward shoot of the RK4 steps from X with the benchmark momenta"}[args.mode]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_match": ttm,
        "time_to_match_curve2d": ttm2,
        "time_to_match_circle_ellipse": ttm3,
        "batched": batched,
        "adjoint": adjoint,
        "shoots": shoots,
        "gpu_ms": {"shoot": shoot_ms, "solve": solve_ms, "factor": factor_ms},
        "records": records,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
