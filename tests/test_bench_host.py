"""Host-side logic of bench.py (no GPU): the single-GPU guard, the roofline
arithmetic of the JSON line on synthetic profiling records, and the serving
latencies by grid size."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode == 2 and "one GPU" in p.stderr


def test_alu_roofline_of_the_walk():
    # 10 launches of 16.7M nodes in 70 ms (timed) and 3 in 18 ms alone, with
    # test counts taken on the device during each set of launches
    nodes = 16_777_216
    walk = lambda k: {"tri_tests": 300.0 * k * nodes, "aabb_tests": 800.0 * k * nodes,
                      "obb_tests": 100.0 * k * nodes, "nodes": k * nodes}
    res = {"dominant": "sdf", "prof": {"launches": 10, "ms": 70.0, "units": 10.0 * nodes},
           "per_kind": {"sdf": {"launches": 3, "ms": 18.0, "units": 3.0 * nodes}},
           "walk_timed": walk(10), "walk_plain": walk(3), "walk_ktz": 4}
    r = bench.roofline(res)
    per_node = 300 * (8.0 / 4 + 37.0) + 800 * (11.0 / 4 + 7.0) + 100 * (17.0 / 4 + 18.0)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == bench.FP32_VALU_TFLOPS
    assert r["avg_launch_us"] == pytest.approx(7000.0)
    assert r["flops_per_node"] == pytest.approx(per_node)
    assert r["achieved"] == pytest.approx(per_node * nodes / 7e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    assert r["frac_unpacked"] == pytest.approx(r["achieved"] / 78.6)
    assert r["tests_per_node"]["triangle"] == pytest.approx(300.0)
    assert r["alone"]["avg_launch_us"] == pytest.approx(6000.0)
    assert r["alone"]["frac"] == pytest.approx(r["frac"] * 7.0 / 6.0)


def test_stale_counter_profiles_are_not_reported(tmp_path, monkeypatch):
    # a counter summary taken on another build of the kernel's source is ignored
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "pmc_sdf_flapping256.txt").write_text("source_sha 0123456789abcdef\ntraffic_bytes_per_launch 5e8\n")
    real = bench.source_sha("paper_2609_20964_amd/csrc/surface.hip")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_sha", lambda rel: real)
    assert bench.load_pmc("sdf") == {}
    (prof / "pmc_sdf_flapping256.txt").write_text(f"source_sha {real}\ntraffic_bytes_per_launch 5e8\n")
    assert bench.load_pmc("sdf")["traffic_bytes_per_launch"] == 5e8


def test_solver_roofline_against_peak_and_copy():
    kinds = {k: {"units": 1e9, "ms": 0.25, "launches": 4} for k in bench.SOLVER_KINDS}
    res = {"solver_kinds": kinds, "solve_ms": [2.0, 2.0]}
    s = bench.solver_hbm(res, copy_gbs=5000.0)
    n = len(bench.SOLVER_KINDS)
    assert s["kernels_GB_s"] == pytest.approx(n * 1e9 / (n * 0.25 * 1e6))
    assert s["phase_GB_s"] == pytest.approx(n * 1e9 / (4.0 * 1e6))
    assert s["kernels_frac"] == pytest.approx(s["kernels_GB_s"] / 8000.0)
    assert s["kernels_frac_of_copy"] == pytest.approx(s["kernels_GB_s"] / 5000.0)
    assert s["phase_ms"] == pytest.approx(2.0)


def test_solver_counter_bytes_from_the_profile(tmp_path, monkeypatch):
    # each kind's bytes are priced by its kernel's counter / algorithmic ratio,
    # from a summary taken on the current solver source only
    real = bench.source_sha("paper_2609_20964_amd/csrc/solver.hip")
    rows = {"k_stencil4<OpPMatvec<false> >": 1.25, "k_vc_pre": 1.5, "k_vc_post<true>": 1.0,
            "k_stencil4<OpResid64<float> >": 1.0, "k_cg_update<false>": 1.0}
    lines = [f"# source_sha {real} (solver.hip)",
             f"# {'kernel':<44} {'fetch_MB':>9} {'write_MB':>9} {'total_MB':>9} {'algorithmic_MB':>15} {'ratio':>6}"]
    for name, r in rows.items():
        lines.append(f"  {name:<44} {100.0 * r - 50:>9.1f} {50.0:>9.1f} {100.0 * r:>9.1f} {100.0:>15.1f} "
                     f"{r:>6.2f}   # a comment")
    path = tmp_path / "pmc_solver_flapping256.txt"
    path.write_text("\n".join(lines) + "\n")
    ratios = bench.solver_counter_ratios(str(path))
    assert ratios == pytest.approx({"sweep": 1.25, "smooth": 1.5, "transfer": 1.0, "resid64": 1.0, "cgupdate": 1.0})
    stale = tmp_path / "stale.txt"
    stale.write_text("\n".join(["# source_sha 0123456789abcdef (solver.hip)"] + lines[1:]) + "\n")
    assert bench.solver_counter_ratios(str(stale)) == {}
    monkeypatch.setattr(bench, "solver_counter_ratios", lambda path=None: ratios)
    kinds = {k: {"units": 1e9, "ms": 0.25, "launches": 4} for k in bench.SOLVER_KINDS}
    s = bench.solver_hbm({"solver_kinds": kinds, "solve_ms": [2.0]})
    assert s["counter_GB_s"] == pytest.approx(s["kernels_GB_s"] * (1.25 + 1.5 + 3.0) / 5)
    assert "counter_GB_s" not in bench.solver_hbm({"solver_kinds": kinds, "solve_ms": [2.0]}, counters=False)


def test_latency_by_grid():
    grids = [64, 256, 64, 128, 64, 256]
    lat = [0.001, 0.030, 0.003, 0.010, 0.002, 0.040]
    out = bench.latency_by_grid(grids, lat)
    assert list(out) == ["64", "128", "256"]
    assert out["64"]["requests"] == 3 and out["64"]["p50_ms"] == pytest.approx(2.0)
    assert out["128"]["p50_ms"] == pytest.approx(10.0) and out["128"]["p99_ms"] == pytest.approx(10.0)
    assert out["256"]["p50_ms"] == pytest.approx(35.0)
    assert out["256"]["p99_ms"] == pytest.approx(30.0 + 0.99 * 10.0)


def test_eikonal_diagnostic_of_exact_and_scaled_distances():
    import numpy as np
    n, h = 48, 1.0 / 48
    z, y, x = np.meshgrid(*(np.arange(n) * h + h / 2,) * 3, indexing="ij")
    phi = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) - 0.3
    e = bench.eikonal(phi, h)
    assert e["within_5pct"] == 1.0 and abs(e["median"] - 1.0) < 1e-3 and e["nodes"] > 1000
    e2 = bench.eikonal(2.0 * phi, h)
    assert e2["within_5pct"] == 0.0 and abs(e2["median"] - 2.0) < 5e-3
