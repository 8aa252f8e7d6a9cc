"""Host logic of bench.py (no GPU): the one-GPU guard, the tile-skipping radius of each cutoff
workload, and the workload table's sizes."""
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("name", [k for k in bench.WORKLOADS if k.endswith("_cut")])
def test_cutoff_radius_is_where_the_kernel_falls_to_eps(name):
    """The conical kernel exp(-r/sigma) and the Gaussian exp(-r^2/sigma^2) equal eps exactly at
    the radius bench.py uses for tile skipping (the bound on the dropped terms scales with it)."""
    spec = bench.WORKLOADS[name][0]
    rc = bench.cutoff_radius(spec)
    s = spec["sigma"]
    g = math.exp(-rc / s) if spec["kernel"] == 0 else math.exp(-(rc / s) ** 2)
    assert g == pytest.approx(spec["eps"], rel=1e-12)


def test_all_pairs_workloads_have_no_cutoff():
    for name, (spec, _) in bench.WORKLOADS.items():
        if not name.endswith("_cut"):
            assert bench.cutoff_radius(spec) == 0.0


def test_workload_sizes():
    """The 3-D sphere at N = 65536 with 100 RK4 steps, the 2-D curve at N = 4096 with 200 and
    the circle -> ellipse at N = 64 with 100."""
    sizes = {name: (spec["n"], spec["steps"]) for name, (spec, _) in bench.WORKLOADS.items() if "n" in spec}
    assert all(v == (65536, 100) for k, v in sizes.items() if k.startswith("sphere3d"))
    assert all(v == (4096, 200) for k, v in sizes.items() if k.startswith("curve2d"))
    assert bench.WORKLOADS["circle_ellipse_f64"][0]["n"] == 64


def test_default_step_is_one_forward_shoot_of_the_sphere():
    a = bench.parse_args([])
    assert a.mode == "shoot" and a.workload == "sphere3d_conon_f64" and a.gpus == 1
    spec, dtype = bench.WORKLOADS[a.workload]
    assert (spec["n"], spec["kernel"], spec["sigma"], spec["steps"], dtype) == (65536, 0, 0.05, 100, 0)


def test_budget_skips_legs_that_do_not_fit():
    b = bench.Budget(bench.time.time() - bench.T_START + 30.0)
    assert b.allows("short", 5.0)
    assert not b.allows("long", 1000.0)
    assert b.skipped == ["long"]


def test_fp32_charges_are_at_most_the_fp64_charges():
    """Single precision drops the exponential's and the square root's refinement steps, so its
    charge per pair is below the double-precision one for every kernel and dimension."""
    for key, s64 in bench.SLOTS_PER_PAIR.items():
        assert bench.SLOTS_PER_PAIR_F32[key] < s64


def test_cpu_baseline_times_one_rk4_step_of_the_workload():
    """The CPU baseline leg runs the oracle on the benchmark's own workload: one whole RK4 step
    when it fits the time target, sampled rows of one evaluation otherwise."""
    import inputs
    pr = inputs.config_sphere3d(600, sigma=0.1)
    p = pr.p_bench()
    r = bench.cpu_baseline(pr, p, target_s=5.0)
    assert r["kind"] == "oracle" and r["unit"] == "pair-interactions/s" and r["value"] > 0
    assert r["sample"].startswith("one RK4 step") and r["cores"] >= 1
    r = bench.cpu_baseline(pr, p, target_s=1e-6)          # too little time: rows instead
    assert "target rows" in r["sample"] and r["value"] > 0
