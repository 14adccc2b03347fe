"""Host-side helpers of bench.py (no GPU)."""

import bench


def test_source_code_ignores_comments_and_blank_lines():
    a = "int f(int x)  // the answer\n{\n\n    /* two\n       lines */\n    return x + 1;\n}\n"
    b = "int f(int x)\n{\n    return x + 1; // done\n}"
    assert bench.source_code(a) == bench.source_code(b) == "int f(int x)\n{\n    return x + 1;\n}"
    assert bench.source_code(a) != bench.source_code(b.replace("+ 1", "+ 2"))


def test_counter_summary_requires_matching_geometry(tmp_path):
    p = tmp_path / "c.txt"
    p.write_text("# comment: not a key\nworkload: poly500\nop_tile: 64 8 125\n"
                 "kernel_source_sha256: %s\nop_traffic_bytes_per_dispatch: 123\n" % bench.kernel_source_hash())
    kv, src = bench._counter_summary(str(p), "poly500", [64, 8, 125])
    assert kv["op_traffic_bytes_per_dispatch"] == "123"
    kv, src = bench._counter_summary(str(p), "poly500", [64, 8, 63])
    assert kv is None and src.startswith("stale")
    kv, src = bench._counter_summary(str(p), "poly300", [64, 8, 125])
    assert kv is None


def test_valu_flops_scale_with_the_z_chunk_only(tmp_path, monkeypatch):
    p = tmp_path / "v.txt"
    p.write_text("workload: poly500\nop_tile: 64 8 125\nfp32_op_tile: 64 8 63\n"
                 "kernel_source_sha256: %s\nfp64_flops_per_dispatch: 6e10\nfp64_mfma_per_dispatch: 0\n"
                 "fp32_flops_per_dispatch: 5.08e10\nfp32_mfma_per_dispatch: 0\n" % bench.kernel_source_hash())
    monkeypatch.setattr(bench, "VALU_COUNTERS", str(p))
    same = bench.measured_valu("poly500", [64, 8, 63], "fp32", 2.0, 500)
    assert same["flops_per_launch"] == 5.08e10 and "scaled" not in same["source"]
    # 500 planes in chunks of 63 compute 508 element layers, in chunks of 125 504
    other = bench.measured_valu("poly500", [64, 8, 125], "fp32", 2.0, 500)
    assert abs(other["flops_per_launch"] - 5.08e10 * 504 / 508) < 1.0 and "scaled" in other["source"]
    assert bench.measured_valu("poly500", [64, 4, 63], "fp32", 2.0, 500)["achieved"] is None
    # 6e10 flops in 3 ms: 20 TFLOP/s of the 78.6 peak
    assert bench.measured_valu("poly500", [64, 8, 125], "fp64", 3.0, 500)["frac"] == round(20.0 / 78.6, 4)


def test_more_than_one_gpu_is_refused():
    """The benchmark runs on one GPU: --gpus above 1 prints why and exits 2,
    before anything touches a device."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_cpu_baseline_reports_both_legs_and_the_extrapolation():
    out = bench.cpu_baseline("eshelby20", 20, 2, 8000 * 8, 123, 60.0)
    assert out["kind"] == "oracle" and out["unit"] == "Gdof*iter/s"
    assert out["serial"]["threads"] == 1 and out["serial"]["value"] > 0 and out["serial"]["iters"] == 2
    assert out["cores"] >= 1 and out["value"] > 0 and out["cpu_model"]
    # 8x the sample's voxels, 123 GPU iterations
    s = out["serial"]
    assert abs(s["extrapolated_time_to_solution_s"] - s["s_per_iter"] * 8 * 123) <= 0.1 + 1e-3 * s["s_per_iter"] * 984
    if "threaded" in out:
        assert out["threaded"]["threads"] > 1 and out["cores"] == out["threaded"]["threads"]


def test_cpu_time_to_solution_solves_every_case():
    """The oracle's own solves of the benchmark problem: every load case to
    the tolerance, serial (and threaded where OpenMP is built), with the GPU
    figures passed through."""
    from paper_2602_07354_amd import synth
    ms = synth.eshelby_inclusion(8)
    out = bench.cpu_time_to_solution(ms, 1e-8, "residual", {"time_to_solution_s": 0.01})
    assert out["cases"] == ms.nrhs and out["gpu"]["time_to_solution_s"] == 0.01
    assert out["serial"]["time_to_solution_s"] > 0 and len(out["serial"]["iters"]) == ms.nrhs
    if "threaded" in out:
        assert out["threaded"]["iters"] == out["serial"]["iters"]
