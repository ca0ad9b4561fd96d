"""Host-side checks of bench.py's contract: one GPU only (a request for more
exits with a message and a nonzero status before touching a GPU), and the
counter-traffic helpers."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_short_kernel_names():
    assert bench._short_kernel("void ttx::k_moved<float, false, 64, 64, 4, 4, false>(ttx::TileArgs<float, float>)") == \
        "k_moved<float, false, 64, 64, 4, 4, false>"
    assert bench._short_kernel("ttx_jit_moved_float_b_64x64_20ec9384") == "ttx_jit_moved_float_b_64x64_20ec9384"


def test_traffic_table_is_keyed_by_the_current_sources():
    """profiles/traffic_counters.json holds the hash of the kernel sources it
    was measured with; bench.py reports counter traffic only while they match."""
    import pytest
    with open(os.path.join(ROOT, "profiles", "traffic_counters.json")) as f:
        tr = json.load(f)
    if tr["source_hash"] != bench.kernel_source_hash():
        pytest.skip("counters predate the current kernel sources (bench.py reports traffic as null)")
    assert 1.9 < tr["scale"]["FETCH_SIZE"] < 2.1 and 0.95 < tr["scale"]["WRITE_SIZE"] < 1.05
    for name, k in tr["kernels"].items():
        assert abs(k["traffic_bytes"] - k["fetch_bytes"] - k["write_bytes"]) <= 1, name   # each rounded


def _fake_full():
    """A result dict shaped like the one bench.py builds (36 cases, every leg)."""
    per_case = [dict(case="4d_f32_p%02d_b0.7" % i, perm=[1, 0, 3, 2], size=[160, 160, 64, 32], dtype="f32",
                     beta=0.7, GBps=5000.0 + i, pct_of_d2d=97.0, us=120.0, kernel="ttx_jit_moved_float_b_64x64_%08x" % i)
                for i in range(36)]
    return dict(
        metric=bench.METRIC, value=4900.0, unit="GB/s", n_gpus=1, steps=20, warmup=5, ms_per_step=3.8,
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32+f64", data="synthetic",
        config=dict(workload="paper-shaped transpositions, ~200 MiB per tensor: 4D/5D/6D x FP32/FP64 x "
                             "(beta=0.7, beta=0), alpha=1.3, 36 cases per step", cases=36,
                    bytes_per_step=18840000000, layout="column-major",
                    entry_point="ttx_plan_execute, one plan per case with its size-specialised kernel "
                                "(ttx_plan_specialise, 36 of 36 compiled in 5.2 s before timing)",
                    parallelism="single GPU"),
        per_call_generic=dict(value=4700.0, pct_of_d2d=92.0, entry_point="ttx_transpose"),
        pct_of_d2d=95.0,
        ceilings={k: dict(GBps=5100.0, GBps_median=5000.0, bytes=1 << 31)
                  for k in ("hipMemcpy_d2d", "copy_kernel", "axpby_f32")},
        per_perm_GBps=dict(min=4400.0, median=4900.0, max=5400.0, weakest="6d_f32_p543210_b0.0",
                           weakest_pct_of_d2d=86.0),
        verification=dict(cases=36, elements_compared=1 << 31, differing_elements=0, max_ulp=0, verified=True,
                          how="every element"),
        roofline=dict(bound="hbm", achieved=4600.0, peak=8000.0, unit="GB/s", frac=0.575, traffic=7.3e8,
                      kernel="ttx_jit_moved_float_b_64x64_20ec9384", launches=20, avg_launch_us=136.9,
                      algorithmic_bytes_per_launch=629233920),
        cpu_baseline=dict(value=21.0, unit="GB/s", cores=16, kind="oracle",
                          sample="all 36 cases of the step, min of 3 runs each, inputs of one GPU call copied "
                                 "from the device",
                          one_thread=dict(value=1.5, unit="GB/s", cores=1, sample="12 cases"),
                          host=dict(logical_cpus=256, usable_cpus=16, model="AMD EPYC 9575F 64-Core Processor",
                                    omp_num_threads="16"),
                          seconds=30.0, per_case=[dict(case=p["case"], GBps=20.0, s=0.03, differing_elements=0)
                                                  for p in per_case]),
        specialised=dict(step_GBps_generic=4600.0, step_GBps_specialised=4880.0, step_GBps_tuned=4850.0,
                         per_case=[dict(case=p["case"]) for p in per_case]),
        side=dict(cases=[dict(case=n, GBps=5000.0, pct_of_d2d=95.0, us=100.0, bytes=1, kernel="k")
                         for n in ("ld_f64_packing_a1.0_b0.0", "awkward_f32_a1.0_b0.0", "literal160_f32_p3210",
                                   "literal24x6_f64_p543210")], shapes_tuned_now=0),
        batched=dict(problems=512, algorithmic_bytes=4230000000,
                     per_call=dict(GBps=1132.0, ms=3.7, launches=512, call_latency_p50_us=20.0,
                                   call_latency_p99_us=80.0),
                     batched=dict(GBps=3218.0, ms=1.3, makespan_p50_ms=1.3, makespan_p99_ms=1.35, grid=1024,
                                  tiles=315000, chunks=8000, variants=12, tuned=512, tune_seconds=3.0,
                                  launch="1 persistent kernel per hipGraph replay"),
                     speedup=2.84),
        served=dict(requests=200000, served=dict(GBps=550.0, p50_us=47.0, p99_us=266.0),
                    sequential=dict(GBps=550.0, p50_us=47.0, p99_us=764.0), throughput_ratio=1.0,
                    mix_check=dict(compared=265, bitwise_mismatches=0),
                    saturated=dict(throughput_ratio=3.4)),
        other_types=dict(cases=[dict(case="6d_c32_p051423", GBps=3671.0, pct_of_d2d=71.5, us=1.0, kernel="k")] * 26,
                         pct_of_d2d_median=95.3, GBps_median=4892.0, GBps_min=3671.0, shapes_tuned_now=0),
        packing=[dict(case="A_f32", GBps=5000.0, pct_of_d2d=88.0, us=1.0, transpositions=1)] * 6,
        contraction=[dict(case="ttgt_%d" % i, m=1600, n=1600, k=1600, panel=32, transposed_a=True,
                          transposed_b=True, ms=0.16, TFLOPs=51.09, gemm_ms=0.122, gemm_TFLOPs=67.4,
                          gemm_frac_of_peak=0.429, rest_ms=0.039, rest_bytes=102400000, rest_GBps=2635.0,
                          rest_pct_of_d2d=50.3, torch_tensordot_ms=0.177, x_torch=1.1) for i in range(3)],
        tuning=dict(table="paper_1607_01249_amd/tune/gfx950.txt", shapes_tuned_now=0, seconds=0.0),
        per_perm=per_case)


def test_printed_line_is_compact_and_complete():
    """The printed line stays far below the 8 KB a log tail keeps and carries
    the headline, the roofline and the CPU baseline (the detail goes to a file)."""
    line = bench.compact_line(_fake_full(), "gpurun_out/bench_detail.json")
    text = json.dumps(line, separators=(",", ":"))
    assert len(text) < 3072, len(text)
    assert set(line["contraction"]) == {"ttgt_0", "ttgt_1", "ttgt_2"}
    assert line["contraction"]["ttgt_0"] == dict(ms=0.16, TFLOPs=51.09, gemm_frac_of_peak=0.429, x_torch=1.1)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "pct_of_d2d", "roofline", "cpu_baseline",
              "verified", "batched", "served"):
        assert k in line, k
    assert "workload" in line["config"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in line["roofline"], k
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in line["cpu_baseline"], k
    assert line["verified"] is True
    assert line["batched"]["x_per_call"] == 2.84 and line["served"]["saturated_x_seq"] == 3.4
    assert line["side_pct_of_d2d"]["literal160"] == 95.0
    assert "per_perm" not in line and "per_case" not in json.dumps(line)


def test_ulp_distance():
    import numpy as np
    x = np.array([1.0, -0.0, 0.0, np.nan, -1.0], dtype=np.float32)
    y = np.array([np.nextafter(np.float32(1.0), np.float32(2.0)), 0.0, 0.0, np.nan, -1.0], dtype=np.float32)
    assert bench._ulp_diff(x, y) == 1
    assert bench._ulp_diff(x[1:], y[1:]) == 0   # -0.0 and +0.0 are equal (the bitwise count tells them apart)
    assert bench._ulp_diff(np.array([-1e-45], np.float32), np.array([1e-45], np.float32)) == 2
    z = np.array([1.0, 2.0], dtype=np.float64)
    assert bench._ulp_diff(z, z) == 0
    assert bench._ulp_diff(np.array([np.float64(1.0)]), np.array([np.nextafter(1.0, 0.0)])) == 1
