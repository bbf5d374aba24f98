#!/usr/bin/env python3
"""Benchmark of the ETD2RKds hot path on one MI355X.

One "step" is one ETD2RKds step (Sec. 3, eq. (11)) of both components over
the whole grid: the stage-1 kernel, 2*d grouped mu-mode-product launches and,
where the last product of the phi_1 operator cannot carry it, a stage-2 kernel.
Default workload: the 3D advective Brusselator on a 256^3 grid (tau = 5e-3,
FP64), with seeded synthetic initial data already resident in HBM.

Prints ONE JSON line with the throughput (grid-point-steps/s), the roofline
position of the dominant kernel (the FP64 MFMA mode product, timed with HIP
events on its own stream inside the timed pass), and the CPU oracle timed on
the host's cores on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 100] [--warmup 5] [--precision f64]

`--workload fhn3d` or `--workload schnakenberg2d` (with --no-extras) puts
another model's workload on the main line, for profiling it alone.

Besides the main line's workload it reports (unless --no-extras): the FP32
and split-BF16 products on the same grid, the 2D Schnakenberg 64^2 and 3D
FitzHugh-Nagumo 128^3 workloads, the 64-instance batched 2D
Schnakenberg workload (grouped plans vs one-by-one), and the serving stream's
p50/p99 latency and throughput (continuous batching vs the plain FP64 path
one request at a time).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point-steps/s at 256³ (FP64 vs split-BF16/FP32) + p50/p99 solve latency"
PEAKS = {  # published MI355X dense peaks
    "f64_mfma_tflops": 78.6,
    "f64_vector_tflops": 78.6,
    "f32_mfma_tflops": 157.3,
    "bf16_mfma_tflops": 2500.0,
    "hbm_gbs": 8000.0,
}
CHIP_CUS = 256   # compute units (the peaks above are for all of them)
MODE_SRC = {"f64": "mode_product_f64.hip", "f32": "mode_product_lowp.hip",
            "bf16x3": "mode_product_lowp.hip", "bf16x2": "mode_product_lowp.hip"}
# BF16 MFMA products per FP32-equivalent product of a split-BF16 precision:
# three parts (hi, mid, lo) take six, two parts (hi, lo) three
SPLIT_PRODUCTS = {"bf16x3": 6, "bf16x2": 3}


def _src_hash(name: str) -> str:
    """Hash of a kernel source's code: line comments and blank lines are dropped,
    so a counter summary stays valid across comment-only edits."""
    path = os.path.join(ROOT, "paper_2307_10684_amd", "csrc", name)
    with open(path, encoding="utf-8") as f:
        lines = [ln.split("//", 1)[0].rstrip() for ln in f]
    code = "\n".join(ln for ln in lines if ln)
    return hashlib.sha256(code.encode()).hexdigest()[:16]


# main workloads: synth builder, default grid side, model description
WORKLOADS = {
    "brusselator3d": ("brusselator_3d", 256,
                      "advective Brusselator (A=1, B=3, Du=1e-3, Dv=5e-3, alpha=0.1*(1,.5,.25))"),
    "fhn3d": ("fhn_3d", 128, "FitzHugh-Nagumo (delta=4, eps=0.1, a1=2, a0=0)"),
    "schnakenberg2d": ("schnakenberg_2d", 64, "Schnakenberg (a=0.1, b=0.9, d=10, gamma=200)"),
}


def _traffic_from_profiles(precision: str, workload: str):
    """HBM bytes per launch of the mode product from the committed counter summary,
    or None if there is none or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"mode_product_{precision}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != _src_hash(MODE_SRC[precision]):
        return None
    # a summary that covers several sources lists them with their hashes
    for item in vals.get("kernel_sources", "").split(","):
        parts = item.split()
        if len(parts) == 2 and _src_hash(os.path.basename(parts[0])) != parts[1]:
            return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _stage_traffic_from_profiles(workload: str, stage1_only: bool):
    """Average HBM bytes per launch of the FP64 stage kernels of a step (stage 1
    alone when the mode product carries stage 2) from the committed counter
    summary, or None (no summary, or stage.hip changed since)."""
    path = os.path.join(ROOT, "profiles", f"stage_kernels_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != _src_hash("stage.hip"):
        return None
    try:
        s1 = float(vals["k_etd_stage1_tile_hbm_bytes_per_launch"])
        if stage1_only:
            return s1
        return 0.5 * (s1 + float(vals["k_etd_stage2_hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    return "unknown"


def _blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def oracle_sample(workload, seed: int, steps: int):
    """The oracle's state after `steps` steps from the seeded initial state (the
    reference the GPU runs are compared against), and the wall time of the last
    steps - 1 of them (the first step is the warm-up)."""
    import oracle as O
    import synth as S
    p = O.problem_from_workload(workload)
    mats = O.precompute(p)
    U, V = S.initial_state(workload, seed)
    U, V = O.etd2rkds_step(U, V, p, mats)  # first touch outside the timing
    t0 = time.perf_counter()
    for _ in range(steps - 1):
        U, V = O.etd2rkds_step(U, V, p, mats)
    return (U, V), time.perf_counter() - t0, (p, mats)


def cpu_baseline(workload, seed: int, steps: int = 5, single_steps: int = 1):
    """The oracle as it stands, timed on the host: `steps - 1` steps with the BLAS
    library on all the threads it takes (the line's value), then `single_steps`
    more on one thread.  Returns the record and the oracle state after `steps`
    steps from the initial state."""
    import oracle as O
    threads = _blas_threads()
    ref, dt, (p, mats) = oracle_sample(workload, seed, steps)
    rec = {
        "value": workload.N * (steps - 1) / dt,
        "unit": "grid-point-steps/s",
        "cores": int(threads),
        "kind": "oracle",
        "cpu_model": _cpu_model(),
        "host_cpus": os.cpu_count(),
        "sample": f"{steps - 1} ETD2RKds steps of {workload.name} after one warm-up step "
                  f"(numpy FP64 oracle, {dt:.1f} s, BLAS threads={threads})",
    }
    if single_steps > 0:
        try:
            from threadpoolctl import threadpool_limits
            U, V = ref
            with threadpool_limits(limits=1):
                t0 = time.perf_counter()
                for _ in range(single_steps):
                    U, V = O.etd2rkds_step(U, V, p, mats)
                dt1 = time.perf_counter() - t0
            rec["single_thread"] = {"value": workload.N * single_steps / dt1, "cores": 1,
                                    "sample": f"{single_steps} ETD2RKds step(s) of {workload.name}, "
                                              f"BLAS on one thread ({dt1:.1f} s)"}
        except Exception as exc:  # pragma: no cover
            rec["single_thread"] = {"error": repr(exc)}
    return rec, ref


def _rel_err(Ud, Vd, ref):
    """max over components of ||gpu - oracle||_inf / ||oracle||_inf."""
    import numpy as np
    Ur, Vr = ref
    shape = Ur.shape
    Ug = Ud.detach().cpu().numpy().reshape(shape, order="F")
    Vg = Vd.detach().cpu().numpy().reshape(shape, order="F")
    return max(float(np.abs(Ug - Ur).max() / np.abs(Ur).max()),
               float(np.abs(Vg - Vr).max() / np.abs(Vr).max()))


def _precision_legs(adr, S, torch, w, steps, seed, oracle_ref, precisions):
    """Throughput of each precision's products on the same workload, and its
    error against the FP64 oracle after the oracle sample's steps."""
    out = {}
    ref_steps, ref_state = oracle_ref if oracle_ref else (0, None)
    for prec in precisions:
        solver = adr.Solver(w, precision=prec)
        U0, V0 = S.initial_state(w, seed)
        Ud, Vd = solver.upload(U0, V0)
        solver.solve(Ud, Vd, 2)                       # warm
        Ud2, Vd2 = solver.upload(U0, V0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.solve(Ud2, Vd2, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err = None
        if ref_state is not None:
            Ue, Ve = solver.upload(U0, V0)
            solver.solve(Ue, Ve, ref_steps)
            torch.cuda.synchronize()
            err = _rel_err(Ue, Ve, ref_state)
            del Ue, Ve
        leg = {"value": w.N * steps / dt, "ms_per_step": 1e3 * dt / steps, "steps": steps,
               "rel_inf_err_vs_oracle": err, "oracle_steps": ref_steps}
        if prec != "f64":
            # a separate pass with HIP events around each launch: the products' roofline
            d = len(w.n)
            adr.adr_timing_enable(steps * (2 * d + 4) + 8)
            solver.solve(Ud, Vd, steps)
            torch.cuda.synchronize()
            n_mode, ms_mode = adr.adr_timing_read(0)
            n_fused, ms_fused = adr.adr_timing_read(3)
            adr.adr_timing_enable(0)
            avg = ms_mode / max(n_mode, 1)
            leg["roofline"] = _lowp_roofline(prec, w, avg, n_mode,
                                             (ms_fused / n_fused) if n_fused else None)
        out[prec] = leg
        del solver, Ud, Vd, Ud2, Vd2
    return out


def _lowp_roofline(prec, w, avg_ms, launches, fused_avg_ms):
    """Roofline of one reduced-precision product launch (both components).
    Algorithmic work: 2 n_mu N flops per component, FP32 operands in and out
    (8 bytes per point per component).  FP32 is bound by the FP32 matrix rate.
    A split-BF16 product runs its flops as `parts` BF16 MFMA products, so its
    matrix-core bound is the BF16 rate divided by that count (in flops of the
    FP32-equivalent work); against the HBM time of its operands it is the
    slower of the two that bounds it."""
    d = len(w.n)
    flops = 2 * 2.0 * (sum(w.n) / d) * w.N
    nbytes = 2 * 2 * 4 * w.N
    tf = flops / (avg_ms * 1e-3) / 1e12
    gbs = nbytes / (avg_ms * 1e-3) / 1e9
    rec = {"kernel": f"mode_product_{prec}", "avg_launch_ms": avg_ms, "launches": launches,
           "flops_per_launch": flops, "algorithmic_bytes_per_launch": nbytes,
           "hbm_gbs": gbs, "fused_launch_avg_ms": fused_avg_ms}
    if prec == "f32":
        rec.update({"bound": "mfma", "achieved": tf, "peak": PEAKS["f32_mfma_tflops"],
                    "unit": "TFLOP/s", "frac": tf / PEAKS["f32_mfma_tflops"]})
        return rec
    parts = SPLIT_PRODUCTS[prec]
    mfma_peak = PEAKS["bf16_mfma_tflops"] / parts          # FP32-equivalent TFLOP/s
    t_mfma = flops / (mfma_peak * 1e12)
    t_hbm = nbytes / (PEAKS["hbm_gbs"] * 1e9)
    if t_mfma >= t_hbm:
        rec.update({"bound": "mfma", "achieved": tf, "peak": mfma_peak, "unit": "TFLOP/s",
                    "frac": tf / mfma_peak,
                    "peak_derivation": f"{PEAKS['bf16_mfma_tflops']} TFLOP/s BF16 / {parts} products"})
    else:
        rec.update({"bound": "hbm", "achieved": gbs, "peak": PEAKS["hbm_gbs"], "unit": "GB/s",
                    "frac": gbs / PEAKS["hbm_gbs"], "tflops_fp32_equivalent": tf})
    return rec


def _whole_step_record(w, steps, launches, ms):
    """The launch that runs every step of a small 2D FP64 problem: its product
    flops (8 sum(n_mu) N per step, FP64 FMAs on the vector units) against the
    FP64 vector peak.  At 4096 points it is bound by the latency of its two grid
    barriers per step, not by arithmetic."""
    flops = 8.0 * sum(w.n) * w.N * steps
    tf = flops / (ms * 1e-3) / 1e12
    # one workgroup of four columns per CU: the share of the chip the launch holds
    cus = -(-int(w.n[1]) // 4)
    own_peak = PEAKS["f64_vector_tflops"] * cus / CHIP_CUS
    return {"kernel": "etd_small2d (all steps in one cooperative launch)", "bound": "alu",
            "launches": launches, "steps": steps, "ms_per_step": ms / steps,
            "achieved": tf, "peak": PEAKS["f64_vector_tflops"], "unit": "TFLOP/s",
            "frac": tf / PEAKS["f64_vector_tflops"], "flops_per_launch": flops / launches,
            "cus": cus, "peak_of_own_cus": own_peak, "frac_of_own_cus": tf / own_peak}


def _workload_legs(adr, S, torch, seed, with_oracle=True):
    """The other two model workloads at one GPU, FP64: the 2D Schnakenberg 64^2
    (launch-bound at 4096 points) and the 3D FitzHugh-Nagumo 128^3, with the mode
    products' position against the FP64 matrix peak.  The 64^2 problem is also
    stepped as a one-problem grouped plan replayed from a HIP graph."""
    out = {}
    # (leg, workload, timed steps, oracle steps: the full configured run of 64^2, a
    # bounded sample of 128^3)
    for name, w, steps, osteps in (("schnakenberg2d_64", S.schnakenberg_2d(64, 400), 400, 100),
                                   ("fhn3d_128", S.fhn_3d(128, 200), 200, 5)):
        solver = adr.Solver(w)
        U0, V0 = S.initial_state(w, seed)
        err = None
        if with_oracle:
            ref, _, _ = oracle_sample(w, seed, osteps)
            Ue, Ve = solver.upload(U0, V0)
            solver.solve(Ue, Ve, osteps)
            torch.cuda.synchronize()
            err = _rel_err(Ue, Ve, ref)
            del Ue, Ve
        Ud, Vd = solver.upload(U0, V0)
        solver.solve(Ud, Vd, 3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.solve(Ud, Vd, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        d = len(w.n)
        adr.adr_timing_enable(steps * (2 * d + 4) + 8)
        solver.solve(Ud, Vd, steps)
        torch.cuda.synchronize()
        n_mode, ms_mode = adr.adr_timing_read(0)
        n_fused, ms_fused = adr.adr_timing_read(3)
        n_whole, ms_whole = adr.adr_timing_read(4)
        n_all, ms_all = adr.adr_timing_read(2)
        adr.adr_timing_enable(0)
        # mode-product flops of a step: 4 Tucker operators, 2 components, 2 n_mu N each
        flops_step = 8.0 * sum(w.n) * w.N
        ms_products = ms_mode + ms_fused
        tf = flops_step * steps / (ms_products * 1e-3) / 1e12 if ms_products > 0 else None
        leg = {"grid": list(w.n), "steps": steps, "value": w.N * steps / dt,
               "ms_per_step": 1e3 * dt / steps,
               "rel_inf_err_vs_oracle": err, "oracle_steps": osteps if with_oracle else None,
               "mode_products": None if tf is None else {
                   "launches_per_step": (n_mode + n_fused) / steps,
                   "ms_per_step": ms_products / steps,
                   "tflops": tf, "peak": PEAKS["f64_mfma_tflops"],
                   "frac": tf / PEAKS["f64_mfma_tflops"]},
               "kernel_ms_per_step": ms_all / steps}
        if n_whole:
            leg["whole_step_kernel"] = _whole_step_record(w, steps, n_whole, ms_whole)
        if name == "schnakenberg2d_64":
            Ub, Vb = solver.upload(U0, V0)
            b = adr.Batch([solver], [(Ub, Vb)], adr.ADR_BATCH_GRAPH)
            b.run(3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.run(steps)
            torch.cuda.synchronize()
            dtg = time.perf_counter() - t0
            b.close()
            leg["graph_plan"] = {"value": w.N * steps / dtg, "ms_per_step": 1e3 * dtg / steps}
        out[name] = leg
        del solver, Ud, Vd
    return out


def _batched_leg(adr, S, torch, steps, seed):
    """The 64-instance batched 2D Schnakenberg workload: grouped plans (FP64 with
    autotuned tiles, FP32), each captured in a graph, against the same instances
    stepped one by one with adr_solve."""
    works = S.batched_schnakenberg_2d(64, steps, seed=seed)
    total = sum(w.N for w in works)
    out = {"workload": "64 x 2D Schnakenberg, sides drawn from {64..512}, tau=1e-3",
           "grid_points": total, "steps": steps}
    init = [S.initial_state(w, seed + 1 + k) for k, w in enumerate(works)]
    for prec in ("f64", "f32"):
        solvers = [adr.Solver(w, precision=prec) for w in works]
        states = [s.upload(*u) for s, u in zip(solvers, init)]
        flags = adr.ADR_BATCH_GRAPH | (adr.ADR_BATCH_AUTOTUNE if prec == "f64" else 0)
        b = adr.Batch(solvers, states, flags)
        b.run(3)                                       # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cfg, graph = b.info()
        b.close()
        out[prec] = {"value": total * steps / dt, "ms_per_step": 1e3 * dt / steps,
                     "tile_cfg_per_mu": cfg[:2], "graph": graph}
        if prec == "f64":
            t0 = time.perf_counter()
            for s, (Ud, Vd) in zip(solvers, states):
                s.solve(Ud, Vd, steps)
            torch.cuda.synchronize()
            dt1 = time.perf_counter() - t0
            out["f64_one_by_one"] = {"value": total * steps / dt1, "ms_per_step": 1e3 * dt1 / steps}
        del solvers, states
    return out


def _serving_leg(S, count, rate, budget_gib, seed, low_rate=None):
    """The serving stream: Poisson arrivals of mixed 2D/3D requests, served by the
    continuous-batching engine (second of two passes over the stream) and, for
    comparison, one at a time by the plain FP64 path, on the same arrival
    times."""
    from paper_2307_10684_amd import serving
    reqs = S.serving_stream(count, rate, seed)
    payload = {r.rid: S.initial_state(r.workload, r.seed) for r in reqs}
    jobs = [serving.Job(r.rid, r.arrival, r.workload, r.workload.steps,
                        lambda k=r.rid: payload[k]) for r in reqs]
    be = serving.GpuBackend("f64")
    eng = serving.Engine(be, budget_bytes=budget_gib << 30, max_active=64, max_chunk=16,
                         lane_bounds=(4e9,), keep_results=True)
    # one untimed pass of the same stream first: device allocations, the
    # matrix-function scratch and the plan-table pool reach their steady sizes
    eng.run(jobs)
    eng.run(jobs)
    _, seq = serving.run_sequential(be, jobs, keep_results=True)
    keys = ("p50_latency_s", "p99_latency_s", "throughput", "makespan_s", "mean_wait_s",
            "peak_active", "peak_bytes", "rounds", "plans_built", "lanes")
    low = None
    if low_rate:
        # the same requests arriving at a rate both paths keep up with: latency
        # without queueing (one pass each; the passes above warmed the allocations)
        lreqs = S.serving_stream(count, low_rate, seed)
        ljobs = [serving.Job(r.rid, r.arrival, r.workload, r.workload.steps,
                             lambda k=r.rid: payload[k]) for r in lreqs]
        eng_low = serving.Engine(be, budget_bytes=budget_gib << 30, max_active=64, max_chunk=16,
                                 lane_bounds=(4e9,), keep_results=False)
        eng_low.run(ljobs)
        _, lseq = serving.run_sequential(be, ljobs, keep_results=False)
        low = {"rate_per_s": low_rate,
               "continuous_batching_f64": {k: eng_low.stats[k] for k in keys},
               "sequential_plain_f64": {k: lseq[k] for k in ("p50_latency_s", "p99_latency_s",
                                                             "throughput", "makespan_s")}}
    return {
        "workload": f"{count} requests, Poisson rate {rate}/s: 50% 2D Schnakenberg 128^2-1024^2, "
                    "25% 3D FHN, 25% 3D advective Brusselator 32^3-192^3, 50-500 steps, "
                    "tau in [1e-4, 5e-3]",
        "budget_gib": budget_gib,
        "grid_point_steps": eng.stats["grid_point_steps"],
        "continuous_batching_f64": {k: eng.stats[k] for k in keys},
        "sequential_plain_f64": {k: seq[k] for k in ("p50_latency_s", "p99_latency_s",
                                                     "throughput", "makespan_s")},
        "throughput_unit": "grid-point-steps/s",
        "below_saturation": low,
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32", "bf16x3", "bf16x2"])
    ap.add_argument("--scheme", default="etd2rkds", choices=["etd2rkds", "lawson2b"])
    ap.add_argument("--workload", default="brusselator3d", choices=sorted(WORKLOADS),
                    help="main workload (the default is the benchmark's; the others are for profiling)")
    ap.add_argument("--n", type=int, default=None,
                    help="grid side of the main workload (default 256 / 128 / 64 for "
                         "brusselator3d / fhn3d / schnakenberg2d)")
    ap.add_argument("--cpu-steps", type=int, default=5,
                    help="oracle sample: steps from the initial state (the first is untimed); "
                         "its final state is the reference of every GPU result")
    ap.add_argument("--cpu-single-steps", type=int, default=1,
                    help="further oracle steps timed with BLAS on one thread")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-extras", action="store_true",
                    help="only the main workload (no reduced-precision, batched or serving legs)")
    ap.add_argument("--lowp-steps", type=int, default=20)
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-low-rate", type=float, default=5.0,
                    help="second arrival rate, below saturation (0: skip)")
    ap.add_argument("--serve-budget-gib", type=int, default=16)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of this many MiB three times "
                         "(reference traffic for hardware byte counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only (the hot path is a single-GPU kernel; "
              "sharding across GPUs is a design note, not implemented). Use --gpus 1.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import paper_2307_10684_amd as adr
    import synth as S

    if args.copy_calibration > 0:
        count = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(count, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            adr.adr_device_copy(src, dst, count)
        torch.cuda.synchronize()
        del src, dst

    builder, n_default, model_text = WORKLOADS[args.workload]
    w = getattr(S, builder)(args.n or n_default)
    d, N = w.d, w.N
    solver = adr.Solver(w, scheme=args.scheme, precision=args.precision)
    U0, V0 = S.initial_state(w, args.seed)
    Ud, Vd = solver.upload(U0, V0)
    U_init, V_init = Ud.clone(), Vd.clone()
    torch.cuda.synchronize()

    # warm-up, then restart from the initial state
    if args.warmup > 0:
        solver.solve(Ud, Vd, args.warmup)
    Ud.copy_(U_init)
    Vd.copy_(V_init)
    torch.cuda.synchronize()

    # ---- timed region: exactly `steps` steps in one adr_solve call
    t0 = time.perf_counter()
    solver.solve(Ud, Vd, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    finite = bool(torch.isfinite(Ud).all().item() and torch.isfinite(Vd).all().item())

    # ---- same steps again with per-launch HIP events (kernel durations)
    launches_per_step = 2 * d + 4
    Ud.copy_(U_init)
    Vd.copy_(V_init)
    torch.cuda.synchronize()
    adr.adr_timing_enable(args.steps * launches_per_step + 8)
    t1 = time.perf_counter()
    solver.solve(Ud, Vd, args.steps)
    torch.cuda.synchronize()
    elapsed_ev = time.perf_counter() - t1
    n_mode, ms_mode = adr.adr_timing_read(0)
    n_stage, ms_stage = adr.adr_timing_read(1)
    n_fused, ms_fused = adr.adr_timing_read(3)
    n_whole, ms_whole = adr.adr_timing_read(4)
    adr.adr_timing_enable(0)

    # ---- the oracle on the host's cores: a bounded, timed sample of the same
    # workload, whose state after `cpu_steps` steps is the reference of every GPU
    # result below (the main path's and each precision's)
    cpu_rec, oracle_ref, parity = None, None, None
    if not args.no_cpu:
        cpu_rec, ref_state = cpu_baseline(w, args.seed, args.cpu_steps, args.cpu_single_steps)
        oracle_ref = (args.cpu_steps, ref_state)
        if args.scheme == "etd2rkds":
            Ud.copy_(U_init)
            Vd.copy_(V_init)
            solver.solve(Ud, Vd, args.cpu_steps)
            torch.cuda.synchronize()
            parity = {"rel_inf_err_vs_oracle": _rel_err(Ud, Vd, ref_state),
                      "steps": args.cpu_steps, "precision": args.precision}
        else:
            oracle_ref = None

    if not args.no_extras:
        del U_init, V_init, Ud, Vd, solver
        torch.cuda.empty_cache()
        others = tuple(p for p in ("f32", "bf16x3", "bf16x2") if p != args.precision)
        extras = {"precisions": _precision_legs(adr, S, torch, w, args.lowp_steps, args.seed,
                                                oracle_ref, others)}
        torch.cuda.empty_cache()
        extras["workloads"] = _workload_legs(adr, S, torch, args.seed, not args.no_cpu)
        torch.cuda.empty_cache()
        extras["batched"] = _batched_leg(adr, S, torch, args.batch_steps, args.seed)
        torch.cuda.empty_cache()
        extras["serving"] = _serving_leg(S, args.serve_requests, args.serve_rate,
                                         args.serve_budget_gib, args.seed,
                                         args.serve_low_rate or None)
    else:
        extras = {}

    ms_per_step = 1e3 * elapsed / args.steps
    value = N * args.steps / elapsed
    mode_avg_ms = ms_mode / max(n_mode, 1)
    # algorithmic work of the plain mode-product launches: 2 d products per step
    # (both components, 2 n_mu N flops each), less the one a launch that carries
    # a stage holds; a plane-pass launch holds two (directions 1 and 2), so the
    # work per launch is the launches' total over their number
    products_plain = 2 * d * args.steps - n_fused
    flops_per_launch = (products_plain * 2 * 2.0 * (sum(w.n) / d) * N / n_mode if n_mode
                        else 2 * 2.0 * (sum(w.n) / d) * N)
    # the product launch of a step whose epilogue also computes a stage (timed apart),
    # 32 B/point more than a plain launch in both cases: FP64 reads the states C_n
    # (16 B) and writes R2 (16 B); reduced precision reads C_n (16 B) and D1 (8 B) and
    # writes FP64 instead of FP32 (8 B)
    fused_avg_ms = ms_fused / n_fused if n_fused else None
    if n_whole and not n_mode:
        # small 2D grids: every step in one launch (stages and products together)
        roof = _whole_step_record(w, args.steps, n_whole, ms_whole)
        roof["avg_launch_ms"] = ms_whole / n_whole
        roof["traffic"] = None
        bytes_per_launch = None
    elif args.precision == "f64":
        achieved = flops_per_launch / (mode_avg_ms * 1e-3) / 1e12
        # read W and write the result for each component (32 B per point), and
        # for the last product of each Tucker operator also the addend (C_n,
        # C_{n2}: 16 B more), averaged over the step's plain launches; the
        # launch that carries stage 2 is counted apart
        plain_per_step = n_mode / max(args.steps, 1)
        fused_per_step = n_fused / max(args.steps, 1)
        bytes_per_launch = 2 * 2 * 8 * N + (2 * 8 * N * (2 - fused_per_step) / plain_per_step
                                            if plain_per_step > 0 else 0.0)
        roof = {"kernel": "mode_product_f64", "bound": "mfma", "achieved": achieved,
                "peak": PEAKS["f64_mfma_tflops"], "unit": "TFLOP/s",
                "frac": achieved / PEAKS["f64_mfma_tflops"],
                "avg_launch_ms": mode_avg_ms, "launches": n_mode,
                "flops_per_launch": flops_per_launch,
                "algorithmic_bytes_per_launch": bytes_per_launch}
    else:
        roof = _lowp_roofline(args.precision, w, mode_avg_ms, n_mode, fused_avg_ms)
        bytes_per_launch = roof["algorithmic_bytes_per_launch"]
    if n_mode:
        roof["tflops"] = flops_per_launch / (mode_avg_ms * 1e-3) / 1e12
        roof["traffic"] = _traffic_from_profiles(args.precision, w.name)
    # the launch that carries stage 2 (FP64): U tiles read W and U_n and write
    # U_{n2}; V tiles read W, V_n, U_{n2} and U_n and write V_{n2}, R_u and R_v
    # (80 B per point); the reduced-precision last product reads W (FP32), the
    # FP64 state and the FP32 first increment and writes the FP64 state
    # (48 B per point, 32 more than a plain FP32 launch)
    if bytes_per_launch is None:
        fused_bytes = None
    elif args.precision == "f64":
        fused_bytes = 80 * N
    else:
        fused_bytes = bytes_per_launch + 32 * N
    roof["fused_launch"] = None if fused_avg_ms is None else {
        "what": ("last product of the phi_1 operator, stage 2 in its epilogue"
                 if args.precision == "f64" else
                 "last product of the phi_2 operator, writes C_n + D1 + D2 in FP64"),
        "launches": n_fused,
        "avg_launch_ms": fused_avg_ms,
        "tflops": 2 * 2.0 * (sum(w.n) / d) * N / (fused_avg_ms * 1e-3) / 1e12,
        "algorithmic_bytes_per_launch": fused_bytes,
        "hbm_gbs": fused_bytes / (fused_avg_ms * 1e-3) / 1e9,
    }
    stage_avg_ms = ms_stage / max(n_stage, 1)
    # algorithmic bytes per point of the stage kernels, averaged over the launches of a step:
    # FP64: stage 1 (read U,V; write R1u,R1v) 32 B, and stage 2 (read U,V,U2,V2; write R2)
    # 48 B unless the last product of the phi_1 operator carries it (then stage 1 only);
    # reduced precision: stage 1 24 B (FP32 R1), stage 2 32 B (FP32 D1 in, R2 out)
    # (the final C_{n+1} = C_n + D1 + D2 is formed by the last mode product)
    stage_per_step = n_stage / max(args.steps, 1)
    if args.precision == "f64":
        stage_bytes = (32.0 if stage_per_step < 1.5 else (32 + 48) / 2) * N
    else:
        stage_bytes = (24 + 32) / 2 * N

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.n), "scheme": args.scheme,
                   "precision": args.precision, "tau": w.tau, "seed": args.seed,
                   "model": model_text},
        "roofline": roof,
        "stage_kernels": None if not n_stage else {
            "bound": "hbm",
            "avg_launch_ms": stage_avg_ms,
            "achieved": stage_bytes / (stage_avg_ms * 1e-3) / 1e9,
            "peak": PEAKS["hbm_gbs"],
            "unit": "GB/s",
            "frac": stage_bytes / (stage_avg_ms * 1e-3) / 1e9 / PEAKS["hbm_gbs"],
            "launches": n_stage,
            "algorithmic_bytes_per_launch": stage_bytes,
            "traffic": (_stage_traffic_from_profiles(w.name, stage_per_step < 1.5)
                        if args.precision == "f64" and args.scheme == "etd2rkds" else None),
        },
        "timing_pass_ms_per_step": 1e3 * elapsed_ev / args.steps,
        "finite": finite,
        "paper_context": "paper (MATLAB, i7-10750H 6 cores): 64^3 Brusselator ETD2RKds 9.1e-3 s/step "
                         "= 2.9e7 grid-point-steps/s",
    }
    if parity is not None:
        line["parity"] = parity
    if extras:
        extras["precisions"][args.precision] = {
            "value": value, "ms_per_step": ms_per_step, "steps": args.steps,
            "rel_inf_err_vs_oracle": parity["rel_inf_err_vs_oracle"] if parity else None,
            "oracle_steps": args.cpu_steps if parity else None}
        line.update(extras)
    if cpu_rec is not None:
        line["cpu_baseline"] = cpu_rec
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
