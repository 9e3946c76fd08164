#!/usr/bin/env python3
"""Benchmark of the WaveHoltz hot path on one MI355X.

One step = one complete Helmholtz solve to a true FP64 WaveHoltz residual of 1e-8
on the 2D workload: unit square, homogeneous Dirichlet, 1024x1024 cells, c = 1,
omega = 100.3, Gaussian source of width 0.02 at a seeded centre, deflated CG with
the 32 analytic sine modes nearest resonance, FP32 stepping with FP64 filter sum,
Krylov and deflation.  Inputs are resident on the GPU before timing starts.

Prints one JSON line: the metric is wave-step throughput (interior points x time
steps of every wave solve in the solve, divided by the solve's wall time), with
the roofline of the dominant kernel (the FP32 leapfrog + filter step) and the CPU
oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "wave-step Gpts/s (HBM roofline %) + time-to-1e-8 residual per Helmholtz solve"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per interior point per time step of the streaming FP32 step
# kernel (c = 1, no forcing): read W^n 4 + W^{n-1} 4, write W^{n+1} 4, V read+write 16
B_PER_PT_STEP_F32 = 28.0
B_PER_PT_STEP_F64 = 40.0
# HBM bytes per dispatch of the K=8 FP32 fused kernel on this grid, from the two
# rocprofv3 counter passes summarised in profiles/hbm_traffic_fused2d_f32_k8_2d1024.md
# (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000 after calibration on a plain copy).  Valid
# only for the kernel source it was taken on.
TRAFFIC = {"kernel": "k_fused2d<float,8,16,false,false>", "k_fuse": 8,
           "src_sha1": "ace13012828772a42fc8ebdd72da1a040fe6b5dc",
           "fetch_kib": 8891.8, "write_kib": 16427.0, "fetch_scale": 2.000, "write_scale": 1.000}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(p, nt, budget_s=12.0):
    """The oracle (scipy CSR leapfrog, FP64) on the same operator: wave solves until
    the time budget is used, reported as wave-step Gpts/s."""
    import numpy as np
    from oracle import discretization as disc, timeparams as tpm, wavesolve as ws
    L = disc.laplacian(2, p.n)
    tp = tpm.time_parameters(p.omega, 1.0 / p.n, 1.0)
    v = disc.to_interior(p.f)
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < budget_s or k == 0:
        v = ws.apply_S(L, v, tp)
        k += 1
    dt = time.perf_counter() - t0
    pts = (p.n - 1) ** 2
    return {"value": pts * tp.nt * k / dt / 1e9, "unit": "Gpts/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} FP64 wave solves (N_t={tp.nt}) of the {p.n}^2 operator with oracle.wavesolve "
                      f"(scipy CSR, one thread) in {dt:.1f} s; host {cpu_model()}, "
                      f"{len(os.sched_getaffinity(0))} cores visible"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 single-solve comparison")
    ap.add_argument("--probe-traffic", action="store_true",
                    help="for hardware-counter runs: a plain 256 MiB device copy, then 5 wave solves "
                         "of the workload's FP32 operator, and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solves of this workload are "
              "single-GPU and nothing here shards across GPUs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2606_31842_amd as wh
    import workloads as wl

    p = wl.config2()
    n = p.n
    pts = (n - 1) ** 2
    f = torch.from_numpy(p.f).cuda()
    if args.probe_traffic:
        # reference copy: 256 MiB read + 256 MiB written, for scaling FETCH_SIZE / WRITE_SIZE
        a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        v = torch.from_numpy(wl.random_nodal(2, n, 1)).cuda()
        for _ in range(5):
            wh.apply_filter(v, p.omega, precision="mixed")
        torch.cuda.synchronize()
        print(json.dumps({"probe": "traffic", "copy_bytes_each_way": a.numel() * 8}), flush=True)
        return
    defl = wh.sine_deflation(2, n, p.omega, 32)
    kw = dict(solver="dcg", defl=defl, precision="mixed", tol=1e-8, max_iters=50000)
    need = wh.workspace_bytes(2, n, wh.params(p.omega, **{k: v for k, v in kw.items() if k != "defl"}), defl)
    wsp = torch.empty(need, dtype=torch.uint8, device="cuda")

    log(f"bench: workload {p.name}, warmup {args.warmup}, steps {args.steps}")
    for i in range(args.warmup):
        u, info = wh.solve(f, p.omega, workspace=wsp, **kw)
        log(f"warmup {i}: {info['ms']:.1f} ms iters {info['iters']} outer {info['outer']} "
            f"f32 {info['wave_solves_f32']} f64 {info['wave_solves']} res {info['true_rel_res']:.2e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        u, info = wh.solve(f, p.omega, workspace=wsp, **kw)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    info = infos[-1]
    nt = info["nt"]
    steps_per_solve = (info["wave_solves"] + info["wave_solves_f32"]) * nt
    value = pts * steps_per_solve / (ms / 1e3) / 1e9
    log(f"timed: {ms:.2f} ms/solve, {steps_per_solve} wave steps/solve, {value:.1f} Gpts/s")

    # error against the oracle's exact solution (DST diagonalisation, c = 1)
    from oracle import discretization as disc
    U = disc.direct_solve_dst(2, n, p.omega, p.f)
    err = float(np.linalg.norm(u.cpu().numpy() - U) / np.linalg.norm(U))

    # roofline of the dominant kernel: the FP32 streaming step, timed on the stream the
    # library launches on (torch's current stream) over whole wave solves
    v = torch.from_numpy(U).cuda()
    out = torch.empty_like(v)
    reps = 20
    wh.apply_filter(v, p.omega, out=out, precision="mixed")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        wh.apply_filter(v, p.omega, out=out, precision="mixed")
    e1.record()
    torch.cuda.synchronize()
    per_solve_ms = e0.elapsed_time(e1) / reps
    filt_gpts = pts * nt / (per_solve_ms / 1e3) / 1e9
    kf = info["k_fuse"]
    # the dominant kernel alone: back-to-back launches of the K-step fused kernel
    # (or the streaming step when K = 1), timed with events on the library's stream
    launch_us = wh.time_step_kernel(v, p.omega, precision="mixed", k_fuse=kf, reps=50) * 1e3
    units = pts * kf                                   # point-steps per launch
    achieved = B_PER_PT_STEP_F32 * units / (launch_us * 1e-6) / 1e9
    log(f"filter: {per_solve_ms:.3f} ms per wave solve ({filt_gpts:.0f} Gpts/s); K={kf} kernel "
        f"{launch_us:.2f} us per launch, {achieved:.0f} GB/s algorithmic")

    extra = {}
    if not args.no_f64:
        kw64 = dict(kw, precision="f64")
        wh.solve(f, p.omega, **kw64)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        u64, i64 = wh.solve(f, p.omega, **kw64)
        torch.cuda.synchronize()
        extra["f64_single_solve"] = {
            "time_to_tol_ms": (time.perf_counter() - ta) * 1e3, "iters": i64["iters"],
            "wave_solves": i64["wave_solves"], "true_rel_res": i64["true_rel_res"],
            "rel_err_vs_oracle": float(np.linalg.norm(u64.cpu().numpy() - U) / np.linalg.norm(U))}

    traffic = None
    src = os.path.join(ROOT, "paper_2606_31842_amd", "csrc", "wh_fused.hip")
    import hashlib
    if kf == TRAFFIC["k_fuse"] and hashlib.sha1(open(src, "rb").read()).hexdigest() == TRAFFIC["src_sha1"]:
        traffic = round(1024 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_scale"] +
                                TRAFFIC["write_kib"] * TRAFFIC["write_scale"]))
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": "2D unit square Dirichlet 1024x1024, c=1, omega=100.3, Gaussian source "
                               "w=0.02 at seeded centre (seed 2), DCG with the 32 sine modes nearest "
                               "resonance, FP32 stepping / FP64 filter+Krylov, true residual 1e-8",
                   "n": n, "omega": p.omega, "n_defl": 32, "solver": "dcg", "precision": "mixed", "tol": 1e-8},
        "time_to_tol_ms": round(ms, 3),
        "solve": {"iters": info["iters"], "outer": info["outer"], "wave_solves_f32": info["wave_solves_f32"],
                  "wave_solves_f64": info["wave_solves"], "nt": nt, "true_rel_res": info["true_rel_res"],
                  "rel_err_vs_oracle": err},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": (f"k_fused2d<float,{kf},16,false,false> ({kf} FP32 leapfrog steps + FP64 filter "
                                "sum per launch)") if kf > 1 else "k_step2d<float,M_MID> (FP32 leapfrog + FP64 filter)",
                     "k_fuse": kf, "bytes_per_pt_step": B_PER_PT_STEP_F32, "pt_steps_per_launch": units,
                     "bytes_per_launch": B_PER_PT_STEP_F32 * units, "launch_us": round(launch_us, 3),
                     "filter_gpts": round(filt_gpts, 2),
                     "hbm_gbs_from_traffic": None if traffic is None else round(traffic / (launch_us * 1e-6) / 1e9, 1)},
        **extra,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(p, nt)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
