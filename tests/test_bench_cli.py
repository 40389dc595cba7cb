"""CPU checks of bench.py's command line: it refuses more than one GPU before touching
any device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def _fake_detail():
    """A detail record with every key a full bench run fills, at full float precision
    (the shape of the real record; the numbers are placeholders)."""
    import random

    rnd = random.Random(7)

    def v():
        return rnd.uniform(1.0, 9.0) * 10 ** rnd.randint(-4, 4) + 1e-9 / 3

    def fw():
        return {"ms_per_step": v(), "mlups": v(), "bytes_per_cell": 216, "hbm_gbs": v(), "hbm_frac": v(),
                "launches": {"one_step": 0, "two_step": 100}, "hbm_moved_gbs": v(), "hbm_moved_frac": v(),
                "ms_per_two_step_launch": v()}

    hist = [[t, v(), v()] for t in range(0, 4001, 250)]
    runs = {k: {"mlups": v(), "kinetic_energy": [[t, v()] for t in range(0, 2001, 100)], "blew_up_at": None,
                "ke_rel_err_final": v(), "ke_rel_err_max": v(), "spectrum_rel_err_max": v(),
                "spectrum_rel_err_median": v(), "u_rel_l2": v()} for k in ("f64", "f32", "f16s", "bf16s")}
    return {
        "forward": {k: fw() for k in ("f32", "f16s", "bf16s", "f32s", "f64")},
        "forward_one_step_kernel": {k: fw() for k in ("f32", "f32s", "f16s")},
        "fp16s_speedup_vs_f32": v(),
        "forward_d3q19": {k: fw() for k in ("f32", "f64", "f16s")},
        "forward_forced": {f"{m}_{s}": fw() for m in ("guo", "shift") for s in ("f32", "f16s")},
        "d2q9_8192": {f"{k}_{s}": fw() for s in ("f32", "f16s", "f64")
                      for k in ("bgk", "bgk_paired", "mrt", "mrt_paired", "mrt_cell", "mrt_cell_paired", "neural_relu",
                                "neural_tanh")},
        "row_pitch": {f"case{i}": fw() for i in range(6)},
        "shard_512x512x64_f16s": {"periodic_step": {"ms": v(), "mlups": v()},
                                  "slab_step_sequential": {"ms": v(), "mlups": v()},
                                  "slab2_step_pair": {"ms_per_two_steps": v(), "mlups": v()}},
        "adjoint": {k: fw() for k in ("f32", "f16s")},
        "adjoint_scatter_form": {k: fw() for k in ("f32", "f16s")},
        "adjoint_forced": {k: fw() for k in ("f32", "f16s")},
        "adjoint_paired": {k: fw() for k in ("f32", "f16s")},
        "adjoint_paired_forced": {k: fw() for k in ("f32", "f16s")},
        "moments_f32": {"ms": v(), "hbm_gbs": v()},
        "tgv2d_64_f64": {"graph_us_per_step": v(), "launch_loop_us_per_step": v()},
        "device_copy": {"gbs": v(), "torch_copy_gbs": v()},
        "accuracy_vs_f64_gpu": {"steps": 1000, "errors": {k: {"u_rel_l2": v(), "ke_rel_err": v()}
                                                          for k in ("f32", "f32s", "f16s", "bf16s")}},
        "workloads": {
            "precision_384": [{"tau": t, "runs": dict(runs)} for t in (0.5015, 0.505)],
            "forcing_128": {"tau": 0.51, "loss_first": v(), "loss_last": v(), "seconds_per_iteration": v(),
                            "loss_curve": [v() for _ in range(30)]},
            "gradient_precision_128": {"runs": {"f64": {"loss": v()},
                                                **{k: {"loss": v(), "cosine_vs_f64": 1 - v() * 1e-9}
                                                   for k in ("f32", "f16s", "bf16s")}}},
            "flow_control_128_2d": [{"kappa": k, "free": {"history": hist}, "restrained": {"history": hist}}
                                    for k in (5e-5, 5e-4, 5e-3)],
            "stability_512": [{"storage": k, "steps": 500, "first_over_threshold": {"step": 350},
                               "history_step_ke_maxspeed_xyz_rowbytes": [[t, v(), v(), 1, 2, 3, 4]
                                                                         for t in range(25, 501, 25)]}
                              for k in ("f16s", "bf16s", "f32s")],
            "adjoint_512": [{"tau": 0.505, "diverged_before_step": 500, "finite_at_step": 450,
                             "f64_check": {"blew_up_at": None}},
                            {"tau": 0.51, "forward_mlups": v(), "tail_forward_mlups": v(), "backward_mlups": v(),
                             "peak_memory_gb": v(), "grad_finite": True}],
        },
    }


def test_bench_line_is_small_and_complete():
    """The printed line stays a few KB (a runner that keeps only the last 9 KB of the
    output, stderr included, still gets it whole) and carries the headline, the
    roofline, the CPU baseline and the summary; the full record goes to a file."""
    import json
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    detail = _fake_detail()
    head = dict(detail["forward"]["f32"])
    cpu = {"value": 4.5, "unit": "MLUPS", "cores": 16, "kind": "oracle",
           "sample": "FP64 torch-CPU oracle, D3Q27 TGV tau=0.51 on 256^3 cells (the full grid), 6 steps (21.3 s)",
           "single_thread_value": 1.7, "single_thread_sample": "64^3 cells, 5 steps (4.1 s)",
           "host": "AMD EPYC 9575F 64-Core Processor, 256 logical CPUs visible, 1500 GiB available"}
    line = bench.summary_line(head, detail, cpu, 200, 10, 3624615676.0, "bench_detail.json")
    text = json.dumps(line, separators=(",", ":"))
    assert len(text) <= 4096, len(text)
    for k in ("metric", "value", "unit", "ms_per_step", "steps", "warmup", "dtype", "roofline", "cpu_baseline",
              "config", "summary", "n_gpus", "higher_is_better", "vs_baseline", "data", "scaling"):
        assert k in line, k
    assert line["config"]["workload"].startswith("D3Q27 BGK Taylor-Green vortex 256^3")
    assert set(line["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic", "moved_frac",
                                     "steps_per_launch"}
    assert line["roofline"]["frac"] == head["hbm_frac"]
    assert line["roofline"]["steps_per_launch"] == 2
    assert line["roofline"]["kernel"].startswith("lbm::step2_kernel")
    assert line["roofline"]["traffic"] == 3624615676.0
    s = line["summary"]
    for k in ("f16s_speedup_vs_f32", "bf16s_speedup_vs_f32", "f16s_u_rel_l2_vs_f64", "adjoint_local_f32_mlups", "adjoint_paired_f16s_mlups",
              "f64_mlups", "d3q19_f32_mlups", "precision_384", "adjoint_512", "one_step_kernel_f32_mlups",
              "one_step_kernel_f32_hbm_frac", "one_step_kernels_f16s_speedup_vs_f32"):
        assert k in s, k
    assert [r["tau"] for r in s["precision_384"]] == [0.5015, 0.505]
    assert [r["tau"] for r in s["adjoint_512"]] == [0.505, 0.51]
    assert json.loads(text) == json.loads(json.dumps(line))


def test_bench_line_without_optional_measurements():
    """--quick: only the headline is measured; the line is still complete."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    head = {"ms_per_step": 0.62, "mlups": 27000.0, "bytes_per_cell": 216, "hbm_gbs": 5800.0, "hbm_frac": 0.725}
    line = bench.summary_line(head, {"forward": {"f32": head}}, None, 50, 5, None, None)
    assert line["value"] == 27000.0 and line["summary"] == {} and line["cpu_baseline"] is None
    assert line["roofline"]["steps_per_launch"] == 1 and line["roofline"]["frac"] == 0.725
