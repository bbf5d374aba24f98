"""Host-side checks of bench.py: the one-GPU contract, the workload table, the
counter summaries it reads for its traffic figures, and the CPU-baseline
record.  Nothing here touches a GPU."""
import os
import subprocess
import sys

import pytest

import bench
import synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("key", sorted(bench.WORKLOADS))
def test_workload_table_builds_its_workloads(key):
    builder, n, model = bench.WORKLOADS[key]
    w = getattr(S, builder)(n)
    assert w.name == f"{key}_{n}"
    assert all(side == n for side in w.n)
    assert model


def test_default_workload_is_the_benchmark_grid():
    builder, n, _ = bench.WORKLOADS["brusselator3d"]
    w = getattr(S, builder)(n)
    assert w.n == (256, 256, 256) and w.tau == 5e-3


def test_source_hash_ignores_comments_and_blank_lines(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2307_10684_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text("int a = 1;  // one\n\n// note\nint b = 2;\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h1 = bench._src_hash("k.hip")
    (csrc / "k.hip").write_text("int a = 1;\n// another note\n\n\nint b = 2;  // two\n")
    assert bench._src_hash("k.hip") == h1
    (csrc / "k.hip").write_text("int a = 1;\nint b = 3;\n")
    assert bench._src_hash("k.hip") != h1


@pytest.mark.parametrize("precision,workload", [
    ("f64", "brusselator3d_256"), ("f32", "brusselator3d_256"), ("bf16x3", "brusselator3d_256"),
    ("bf16x2", "brusselator3d_256"),
    ("f64", "fhn3d_128")])
def test_committed_counter_summaries_match_the_kernel_sources(precision, workload):
    # a summary taken before the kernel's code last changed is ignored by bench.py
    # (traffic null); the committed ones must be current
    traffic = bench._traffic_from_profiles(precision, workload)
    assert traffic is not None and traffic > 0


def test_committed_stage_summary_matches_the_kernel_source():
    assert bench._stage_traffic_from_profiles("brusselator3d_256", True) is not None


def test_cpu_baseline_record():
    import numpy as np
    import oracle as O
    w = S.schnakenberg_2d(16, 3)
    rec, ref = bench.cpu_baseline(w, 0, steps=3, single_steps=1)
    assert rec["kind"] == "oracle" and rec["unit"] == "grid-point-steps/s"
    assert rec["value"] > 0 and rec["cores"] >= 1
    assert "schnakenberg2d_16" in rec["sample"] and rec["cpu_model"]
    assert rec["single_thread"]["cores"] == 1 and rec["single_thread"]["value"] > 0
    # the reference state is the oracle's after exactly `steps` steps
    U0, V0 = S.initial_state(w, 0)
    U, V = O.solve(U0, V0, O.problem_from_workload(w), 3)
    assert np.array_equal(ref[0], U) and np.array_equal(ref[1], V)


def test_reduced_precision_roofline_bounds():
    # FP32: the FP32 matrix rate.  Split BF16 at n = 256: six products (three
    # parts) take 6 x 2n flops at 2.5 PFLOP/s, longer than moving the FP32
    # operands at 8 TB/s, so the matrix cores bound it (at 2500/6 TFLOP/s of
    # FP32-equivalent work); three products (two parts) take less time than the
    # operands' traffic, so HBM bounds them
    w = S.brusselator_3d()
    r32 = bench._lowp_roofline("f32", w, 0.160, 100, None)
    assert r32["bound"] == "mfma" and r32["peak"] == bench.PEAKS["f32_mfma_tflops"]
    assert abs(r32["achieved"] - 17.179869184e9 / 0.160e-3 / 1e12) < 1e-9
    r3 = bench._lowp_roofline("bf16x3", w, 0.085, 100, None)
    assert r3["bound"] == "mfma" and abs(r3["peak"] - 2500.0 / 6) < 1e-9
    assert abs(r3["frac"] - 17.179869184e9 / 0.085e-3 / 1e12 / (2500.0 / 6)) < 1e-9
    r2 = bench._lowp_roofline("bf16x2", w, 0.085, 100, None)
    assert r2["bound"] == "hbm" and r2["peak"] == bench.PEAKS["hbm_gbs"]
    assert 0 < r2["frac"] < 1


def test_whole_step_record():
    # the 64^2 FP64 step runs as one launch: its record prices the products'
    # 8 sum(n_mu) N flops per step against the FP64 vector peak
    w = S.schnakenberg_2d(64, 10)
    rec = bench._whole_step_record(w, 400, 1, 4.0)
    flops = 8.0 * 128 * 4096 * 400
    assert rec["bound"] == "alu" and rec["peak"] == bench.PEAKS["f64_vector_tflops"]
    assert abs(rec["achieved"] - flops / 4e-3 / 1e12) < 1e-12
    assert abs(rec["frac"] - rec["achieved"] / 78.6) < 1e-15
    assert abs(rec["ms_per_step"] - 0.01) < 1e-15
    # 64 columns, four per workgroup: 16 of the 256 CUs
    assert rec["cus"] == 16
    assert abs(rec["frac_of_own_cus"] - rec["achieved"] / (78.6 * 16 / 256)) < 1e-12
