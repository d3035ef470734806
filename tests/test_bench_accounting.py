"""The benchmark's FLOP model reproduces the paper's per-element FLOP table exactly."""
import json
import os

import bench

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_flops_table.json")


def test_flop_model_matches_paper_table():
    g = json.load(open(GOLD))
    for p, f, fd in zip(g["p"], g["flops_per_element"], g["flops_per_dof"]):
        assert bench.flops_per_element(p) == f
        assert round(bench.flops_per_element(p) / (3 * p ** 3)) == fd


def test_algorithmic_bytes():
    assert bench.algorithmic_bytes(100, 10, 8) == 16 * 100 + 96 * 10
    assert bench.algorithmic_bytes(100, 10, 4) == 8 * 100 + 48 * 10


def test_multi_gpu_request_exits():
    assert bench.main(["--gpus", "2"]) == 2


def _fake_result():
    """A full result of the shape bench.main builds (values arbitrary, lengths realistic)."""
    ps = (1, 2, 4, 6, 8)
    long = "x" * 300
    rate = {"gdofs": 40.123456, "gdofs_hot": 41.2, "us": 100.0, "tflops": 25.0, "frac_alu_peak": 0.3181,
            "frac_alu_measured": 0.38, "gbs": 700.0, "frac_hbm": 0.08, "N": 4260531}
    solve = {"rc": 0, "setup_s": 0.01, "solve_s": 0.0573, "iters": 18, "outer": 0, "rel_res_true": 9.9e-9,
             "levels": 6, "N": 8124675, "err_vs_f64_energy": 1e-9, "time_vs_f64": 0.8}
    serve = {"solves": 512, "failed": 0, "makespan_s": 18.3, "solves_per_s": 27.9, "p50_latency_s": 0.104,
             "p99_latency_s": 0.479, "mean_iters": 14.2, "max_rel_res": 9.9e-9}
    return {
        "metric": "PA apply GDoF/s at p=1..8 (FP64 vs FP32); GMG-PCG solves/s + p99 latency",
        "value": 31.1234, "unit": "GDoF/s", "n_gpus": 1, "steps": 20, "warmup": 5, "ms_per_step": 0.6912,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": long, "dofs": {p: 4260531 for p in ps}, "parallelism": "single GPU"},
        "step_per_p_gdofs": {p: 40.123 for p in ps},
        "roofline": {"bound": "alu", "achieved": 42.5, "peak": 78.6, "unit": "TFLOP/s", "frac": 0.5407,
                     "traffic": 335789264, "kernel": bench.apply_kernel_names(1), "flops_per_launch": 9824716800,
                     "algorithmic_bytes_per_launch": 200876736, "hbm_gbs": 870.1, "launch_us": 228.61,
                     "source_hash": "0123456789abcdef", "measured_peak": 66.1, "frac_measured": 0.64},
        "ceilings": {"fma_f64_tflops": 66.1, "fma_f32_tflops": 75.0, "copy_gbs": 5100.0},
        "sweep": {p: {"f64": dict(rate), "f32": dict(rate)} for p in range(1, 9)},
        "ablation": {"workload": long, **{f"p{p}": {"x": long} for p in (1, 2, 4, 8)}},
        "solve": {"workload": long, **{f"p{p}": {"f64": dict(solve), "f32_ir": dict(solve),
                                                "f32_prec": dict(solve)} for p in (4, 6, 8)},
                  "p8_qpoint": {"workload": long, "f64": dict(solve), "f32_prec": dict(solve)}},
        "serve": {"requests": 512, **{m: dict(serve) for m in ("f32_ir", "f32_prec", "f64")}},
        "cpu_baseline": {"value": 0.00312345678, "unit": "GDoF/s", "cores": 1, "host_cores": 16,
                         "cpu_model": "AMD EPYC 9575F 64-Core Processor" + " " * 40, "kind": "oracle",
                         "value_1thread": 0.0031, "sample": long,
                         "per_p": {p: {"gdofs": 0.00312345678, "t_apply_s": 0.2} for p in ps}},
    }


def test_summary_line_is_short_and_complete():
    s = bench.compact_summary(_fake_result())
    line = json.dumps(s, separators=(",", ":"))
    assert len(line) < 2048, len(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in s, k
    assert "workload" in s["config"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in s["roofline"], k
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in s["cpu_baseline"], k
    assert set(s["sweep_gdofs"]["f64"]) == {str(p) for p in range(1, 9)}
    assert json.loads(line) == s
