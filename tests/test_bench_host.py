"""Host-side logic of bench.py: the counter-profile lookup behind `roofline.traffic` (used only
while the kernel sources hash to the profile's), the roofline object's arithmetic, the kernel
naming, and the single-GPU guard.  No GPU needed."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def current_sha():
    m = hashlib.sha256()
    for f in bench.STEP_SOURCES:
        m.update(open(os.path.join(ROOT, f), "rb").read())
    return m.hexdigest()


def write_profile(path, sha, nbytes):
    with open(path, "w") as f:
        f.write("# summary\n\nMachine-readable:\n\n"
                f"    traffic_bytes_per_launch: {nbytes}\n    source_sha256: {sha}\n")


def test_traffic_is_read_only_while_the_sources_match(tmp_path, monkeypatch):
    good, stale = tmp_path / "good.md", tmp_path / "stale.md"
    write_profile(good, current_sha(), 1234567)
    write_profile(stale, "0" * 64, 1234567)
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", {"k_good": str(good), "k_stale": str(stale),
                                                    "k_missing": str(tmp_path / "none.md")})
    assert bench.measured_traffic("k_good") == 1234567
    assert bench.measured_traffic("k_stale") is None
    assert bench.measured_traffic("k_missing") is None
    assert bench.measured_traffic("k_unknown") is None


def test_committed_profiles_name_the_roofline_kernels():
    for kernel, path in bench.TRAFFIC_PROFILES.items():
        assert os.path.exists(path), path
        assert kernel in ("tb3_step_kernel<float,float,true>", "tb2_step_kernel<float,float,true>",
                          "step_kernel<float,float,true>")


def test_roofline_object_of_a_fused_run(monkeypatch):
    monkeypatch.setattr(bench, "measured_traffic", lambda k: 2_000_000_000)
    nodes = 4096 * 4096
    ms = 0.25                                  # per step; a launch makes two
    run = {"ms": ms, "achieved": bench.BYTES_PER_NODE_FP32 * nodes / (ms * 1e-3) / 1e9,
           "shape": (2, 0, 6, 11611), "kernel": bench.kernel_name("fp32", (2, 0, 6, 11611)),
           "nodes": nodes}
    o = bench.roofline_obj(run)
    assert o["kernel"] == "tb2_step_kernel<float,float,true>" and o["steps_per_launch"] == 2
    assert abs(o["launch_ms"] - 0.5) < 1e-12 and o["rows_per_segment"] == 6
    assert abs(o["frac"] - run["achieved"] / 8000.0) < 1e-4 and o["bound"] == "hbm"
    assert o["traffic"] == 2_000_000_000 and abs(o["measured_hbm_GBps"] - 4000.0) < 0.1
    # the launch's own minimum: 120 B per node once, over the launch (two updates)
    assert o["own_min_bytes_per_launch"] == 120 * nodes
    assert abs(o["frac_own_min"] - 120 * nodes / 0.5e-3 / 8e12) < 1e-4
    assert abs(o["frac_measured_hbm"] - 0.5) < 1e-4
    assert abs(o["traffic_vs_own_min"] - 2e9 / (120 * nodes)) < 1e-3


def test_kernel_names():
    assert bench.kernel_name("fp32", (1, 0, 0, 1)) == "step_kernel<float,float,true>"
    assert bench.kernel_name("fp32_f64", (2, 0, 12, 5)) == "tb2_step_kernel<float,double,true>"
    assert bench.kernel_name("fp32", (3, 0, 16, 4608)) == "tb3_step_kernel<float,float,true>"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "exactly one GPU" in r.stderr
