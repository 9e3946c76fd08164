#!/usr/bin/env python3
"""Benchmark of the WaveHoltz hot path on one MI355X.

One step = one batched solve of 256 2D Helmholtz problems to a true FP64 WaveHoltz
residual of 1e-8 each: 64 problems on each of 128^2, 256^2, 512^2 and 1024^2 cells
(unit square, homogeneous Dirichlet, c = 1), omega ~ U(10, 80) kept off the discrete
resonances, Gaussian sources omega^2 exp(-omega^2 r^2) at seeded centres; deflated CG with
the floor(1.5 omega) sine modes nearest omega^2 per problem, FP32 stepping with FP64
filter sum, Krylov and deflation, rounds replayed from hipGraphs.  Inputs are resident on
the GPU before timing starts.

Prints one JSON line: the metric is wave-step throughput (interior points x time steps of
every wave solve of the batch, divided by the batch's wall time), with the roofline of the
dominant kernel (the batched FP32 work kernel), the same problems in the FP64 single-solve
forms and in batched mixed CG for comparison, and the CPU oracle timed on a bounded sample
together with every solution's error against the oracle's direct solve.  Other workloads:
--workload cfg1 | cfg2 | cfg3 | cfg5 | solvers | ndsweep.
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
# fused-form algorithmic bytes per interior point per launch of a K-step FP32 kernel (no forcing):
# state pair in 4 + 4, state pair out 4 + 4, V read + write 8 + 8
B_FUSED_F32 = 32.0
# HBM KiB per dispatch (FETCH_SIZE, WRITE_SIZE) of the tagged batch work kernel on the config-4
# batch, from the two counter passes in profiles/hbm_traffic_batch_tile_cfg4.md, with the copy-kernel
# scale factors; valid only for the kernel sources it was taken on (sha1 over the three files)
BATCH_TRAFFIC = {"src_sha1": "77f221ac8450026321c4cc81a015087f729457f0", "fetch_scale": 2.0, "write_scale": 1.0,
                 "kib": [744030.1, 1410878.1]}
# HBM KiB per dispatch (FETCH_SIZE, WRITE_SIZE) of every FP32 temporally blocked kernel
# variant "K,R,NW" on this grid, from the two rocprofv3 counter passes summarised in
# profiles/hbm_traffic_fused2d_f32_2d1024.md (scaled by FETCH x 2.000, WRITE x 1.000 from a
# plain copy).  Valid only for the kernel source it was taken on.
TRAFFIC = {"src_sha1": "e20c1609c19597223bdf79e5167b888778df7d6f", "fetch_scale": 2.000, "write_scale": 1.000,
           "kib": {"2,8,4": [8415.0, 16408.0], "2,8,8": [8498.4, 16444.9], "2,16,4": [8533.9, 16438.6],
                   "3,8,4": [8404.2, 16384.3], "3,8,8": [8551.1, 16440.4], "3,16,4": [8591.1, 16436.2],
                   "4,8,4": [8532.1, 16405.0], "4,8,8": [8616.1, 16437.0], "4,16,4": [8654.6, 16435.8],
                   "6,8,4": [8621.4, 16394.0], "6,8,8": [8673.4, 16415.7], "6,16,4": [8725.4, 16411.9],
                   "8,8,4": [8715.2, 16384.4], "8,8,8": [8849.8, 16427.0], "8,16,4": [8905.8, 16427.3]}}


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


def cpu_baseline(p, nt, budget_s=12.0, wave_solves=0, direct=True):
    """The oracle (scipy CSR leapfrog, FP64) on the same operator: wave solves until
    the time budget is used, reported as wave-step Gpts/s.  Beside it, the time the
    oracle would take to the tolerance (extrapolated from the wave-solve count) and
    two direct solves of the same discrete problem on one core: scipy's sparse LU and
    the oracle's sine-transform solve."""
    from oracle import discretization as disc, timeparams as tpm, wavesolve as ws
    L = disc.laplacian(2, p.n)
    tp = tpm.time_parameters(p.omega, 1.0 / p.n, 1.0)
    v = disc.to_interior(p.f)
    with _one_thread():
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < budget_s or k == 0:
            v = ws.apply_S(L, v, tp)
            k += 1
        dt = time.perf_counter() - t0
    pts = (p.n - 1) ** 2
    out = {"value": pts * tp.nt * k / dt / 1e9, "unit": "Gpts/s", "cores": 1, "kind": "oracle",
           "sample": f"{k} FP64 wave solves (N_t={tp.nt}) of the {p.n}^2 operator with oracle.wavesolve "
                     f"(scipy CSR, one thread) in {dt:.1f} s; host {cpu_model()}, "
                     f"{len(os.sched_getaffinity(0))} cores visible",
           "s_per_wave_solve": dt / k}
    if wave_solves:
        # the oracle's WaveHoltz iteration needs the same number of wave solves as the
        # library's to reach the tolerance; its time is that count times the measured rate
        out["extrapolated_time_to_tol_s"] = round(dt / k * wave_solves, 1)
        out["extrapolated_from_wave_solves"] = wave_solves
    if direct:
        out["direct_splu"] = direct_splu(2, p.n, p.omega, p.f)
        t0 = time.perf_counter()
        disc.direct_solve_dst(2, p.n, p.omega, p.f)
        out["direct_dst_s"] = round(time.perf_counter() - t0, 3)
    return out


def _one_thread():
    """BLAS pools limited to one thread for the single-core oracle timings."""
    from threadpoolctl import threadpool_limits
    return threadpool_limits(1)


def oracle_cg_solve(dim, n, omega, f_nodal, tol, c2=None, c_max=1.0):
    """The oracle's FP64 WaveHoltz CG on one problem, one thread: (iterations, N_t, seconds)."""
    from oracle import discretization as disc, krylov as kr, timeparams as tpm, wavesolve as ws
    with _one_thread():
        t0 = time.perf_counter()
        L = disc.laplacian(dim, n, c2)
        tp = tpm.time_parameters(omega, 1.0 / n, c_max)
        b = ws.rhs(L, disc.to_interior(f_nodal), tp)
        _, info = kr.cg(lambda v: ws.apply_A(L, v, tp), b, tol=tol, maxit=100000)
        return info["iters"], tp.nt, time.perf_counter() - t0


def _oracle_cg_job(args):
    return oracle_cg_solve(*args)


def direct_splu(dim, n, omega, f_nodal, c2=None):
    """scipy's sparse LU of the same discrete Helmholtz matrix, one thread."""
    import numpy as np
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    from oracle import discretization as disc
    with _one_thread():
        L = disc.laplacian(dim, n, c2)
        A = (L + omega ** 2 * sp.identity(L.shape[0])).tocsc()
        b = disc.to_interior(f_nodal)
        t0 = time.perf_counter()
        lu = sla.splu(A)
        t1 = time.perf_counter()
        x = lu.solve(b)
        t2 = time.perf_counter()
        return {"factor_s": round(t1 - t0, 3), "solve_s": round(t2 - t1, 4), "lu_nnz": int(lu.L.nnz + lu.U.nnz),
                "rel_res": float(np.linalg.norm(b - A @ x) / np.linalg.norm(b)),
                "note": "scipy SuperLU of the same discrete Helmholtz matrix, one thread"}


def run_cfg2(args, np, torch, wh, wl):
    """Single 2D 1024^2 solve, c = 1, omega = 100.3, mixed DCG with the 32 sine modes nearest
    resonance, true residual 1e-8 (the previous benchmark line, kept as an extra workload)."""
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
    # steps per launch and block shape fixed at the autotuner's pick for this grid (K = 8
    # with 8 rows x 8 waves; K = 6 is 3 % slower over a whole solve), so that the bench
    # line and a profiled run of it time the same kernel
    kfix = dict(k_fuse=8, k_shape=1)
    kw = dict(solver="dcg", defl=defl, precision="mixed", tol=1e-8, max_iters=50000, **kfix)
    need = wh.workspace_bytes(2, n, wh.params(p.omega, **{k: v for k, v in kw.items() if k != "defl"}), defl)
    wsp = torch.empty(need, dtype=torch.uint8, device="cuda")

    log(f"bench: workload {p.name}, warmup {args.warmup}, steps {args.steps}")
    for i in range(args.warmup):
        u, info = wh.solve(f, p.omega, workspace=wsp, **kw)
        log(f"warmup {i}: {info['ms']:.1f} ms iters {info['iters']} outer {info['outer']} "
            f"f32 {info['wave_solves_f32']} f64 {info['wave_solves']} res {info['true_rel_res']:.2e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, step_s = [], []
    for i in range(args.steps):
        ts = time.perf_counter()
        u, info = wh.solve(f, p.omega, workspace=wsp, **kw)
        infos.append(info)
        step_s.append(time.perf_counter() - ts)   # each solve ends in a host readback
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    info = infos[-1]
    nt = info["nt"]
    steps_per_solve = (info["wave_solves"] + info["wave_solves_f32"]) * nt
    value = pts * steps_per_solve / (ms / 1e3) / 1e9
    log(f"timed: {ms:.2f} ms/solve, {steps_per_solve} wave steps/solve, {value:.1f} Gpts/s")

    # accuracy: the library's Helmholtz residual ||f - (L_h + omega^2) u|| / ||f||
    # (element-wise parity against the oracle is the tests' job)
    hres = wh.helmholtz_residual(u, f, p.omega)

    # roofline of the dominant kernel: the FP32 streaming step, timed on the stream the
    # library launches on (torch's current stream) over whole wave solves
    v = u.clone()
    out = torch.empty_like(v)
    reps = 20
    wh.apply_filter(v, p.omega, out=out, precision="mixed", **kfix)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        wh.apply_filter(v, p.omega, out=out, precision="mixed", **kfix)
    e1.record()
    torch.cuda.synchronize()
    per_solve_ms = e0.elapsed_time(e1) / reps
    filt_gpts = pts * nt / (per_solve_ms / 1e3) / 1e9
    kf = info["k_fuse"]
    # the dominant kernel alone: back-to-back launches of the K-step fused kernel
    # (or the streaming step when K = 1), timed with events on the library's stream
    launch_ms, kshape = wh.time_step_kernel(v, p.omega, precision="mixed", reps=50, shape=True, **kfix)
    launch_us = launch_ms * 1e3
    if kshape["k"] != kf:
        log(f"note: the timed kernel uses K={kshape['k']}, the solve used K={kf}")
        kf = kshape["k"]
    units = pts * kf                                   # point-steps per launch
    achieved = B_PER_PT_STEP_F32 * units / (launch_us * 1e-6) / 1e9
    log(f"filter: {per_solve_ms:.3f} ms per wave solve ({filt_gpts:.0f} Gpts/s); K={kf} kernel "
        f"{launch_us:.2f} us per launch, {achieved:.0f} GB/s algorithmic")

    # the box's attainable HBM rate: a plain 1 GiB device-to-device copy (read + write)
    ca = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    e0.record()
    for _ in range(10):
        cb.copy_(ca)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * ca.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del ca, cb
    log(f"copy: {copy_gbs:.0f} GB/s")

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
            "helmholtz_rel_res": wh.helmholtz_residual(u64, f, p.omega)}

    traffic = None
    src = os.path.join(ROOT, "paper_2606_31842_amd", "csrc", "wh_fused_kernel.h")
    import hashlib
    key = f"{kf},{kshape['rows']},{kshape['waves']}"
    if key in TRAFFIC["kib"] and hashlib.sha1(open(src, "rb").read()).hexdigest() == TRAFFIC["src_sha1"]:
        fk, wk = TRAFFIC["kib"][key]
        traffic = round(1024 * (fk * TRAFFIC["fetch_scale"] + wk * TRAFFIC["write_scale"]))
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": "2D unit square Dirichlet 1024x1024, c=1, omega=100.3, Gaussian source "
                               "w=0.02 at seeded centre (seed 2), DCG with the 32 sine modes nearest "
                               "resonance, FP32 stepping / FP64 filter+Krylov, true residual 1e-8",
                   "n": n, "omega": p.omega, "n_defl": 32, "solver": "dcg", "precision": "mixed", "tol": 1e-8,
                   "k_fuse": kfix["k_fuse"], "block": "8 rows x 8 waves"},
        "time_to_tol_ms": round(ms, 3),
        "ms_per_step_min_median": [round(min(step_s) * 1e3, 3), round(sorted(step_s)[len(step_s) // 2] * 1e3, 3)],
        "solve": {"iters": info["iters"], "outer": info["outer"], "wave_solves_f32": info["wave_solves_f32"],
                  "wave_solves_f64": info["wave_solves"], "nt": nt, "true_rel_res": info["true_rel_res"],
                  "helmholtz_rel_res": hres},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": (f"k_fused2d<float,{kf},{kshape['rows']},{kshape['waves']},false,false,0> ({kf} FP32 "
                                "leapfrog steps + FP64 filter sum per launch)") if kf > 1
                               else "k_step2d<float,M_MID> (FP32 leapfrog + FP64 filter)",
                     "k_fuse": kf, "bytes_per_pt_step": B_PER_PT_STEP_F32, "pt_steps_per_launch": units,
                     "bytes_per_launch": B_PER_PT_STEP_F32 * units, "launch_us": round(launch_us, 3),
                     "filter_gpts": round(filt_gpts, 2),
                     "hbm_gbs_from_traffic": None if traffic is None else round(traffic / (launch_us * 1e-6) / 1e9, 1),
                     "traffic_frac_of_peak": None if traffic is None else
                     round(traffic / (launch_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "copy_gbs": round(copy_gbs, 1),
                     "traffic_frac_of_copy": None if traffic is None else
                     round(traffic / (launch_us * 1e-6) / 1e9 / copy_gbs, 4)},
        **extra,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(p, nt, wave_solves=steps_per_solve // nt, direct=not args.no_direct)
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 single-solve comparisons")
    ap.add_argument("--no-direct", action="store_true",
                    help="cfg2: skip the CPU direct solves (scipy sparse LU, about 25 s)")
    ap.add_argument("--workload", default="cfg4",
                    choices=["cfg1", "cfg2", "cfg3", "cfg4", "cfg5", "solvers", "ndsweep", "order4"],
                    help="cfg4 (default) is the benchmark line: 256 batched 2D solves; the others report "
                         "the remaining workloads (2D 64^2 FP64 CG; 2D 1024^2 single mixed DCG solve; 3D 256^3 "
                         "variable c; 513^2 adjoint gradient; the config-2 problem by every solver; "
                         "iterations against omega for two deflation-size rules; fourth-order stepping rates)")
    ap.add_argument("--max-iters", type=int, default=0, help="iteration cap (cfg3, solvers)")
    ap.add_argument("--omegas", default="5:30", help="ndsweep: first:last (step 1) or a comma list")
    ap.add_argument("--runs", default="", help="solvers: comma-separated subset of the run names "
                                               "(cg, dcg_nd8, dcg_nd32, dcg_nd64, devd_cg_nd32, "
                                               "devd_fpi_nd32, gmres, agmres_nd32, bicgstab, "
                                               "abicgstab_nd32, agmres_nd32_dense, agmres_nd32_factored)")
    ap.add_argument("--per-size", type=int, default=64, help="problems per grid size (cfg4)")
    ap.add_argument("--fd-directions", type=int, default=20,
                    help="cfg5: random directions of the central-difference check (0: none)")
    ap.add_argument("--no-cg", action="store_true", help="cfg4: skip the batched mixed CG comparison run")
    ap.add_argument("--probe-traffic", action="store_true",
                    help="for hardware-counter runs: a plain 256 MiB device copy, then the workload's "
                         "dominant kernel (cfg4: the batched FP32 work kernel, 5 launches; cfg3: the "
                         "autotuner's trials and the timed 3D stepping kernels, no solves), and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solves of this workload are "
              "single-GPU and nothing here shards across GPUs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2606_31842_amd as wh
    import workloads as wl

    if args.workload != "cfg4":
        print(json.dumps(EXTRA[args.workload](args, np, torch, wh, wl)), flush=True)
        return

    probs = wl.config4(per_size=args.per_size)
    fs = [torch.from_numpy(q.f).cuda() for q in probs]
    nds = [int(math.floor(1.5 * q.omega)) for q in probs]
    batch = [(f, q.omega) for f, q in zip(fs, probs)]
    K = 8
    kw = dict(solver="dcg", precision="mixed", tol=1e-8, k_fuse=K, max_iters=10000)
    wsp = torch.empty(wh.batch_workspace_bytes(batch, nds, **kw), dtype=torch.uint8, device="cuda")
    if args.probe_traffic:
        a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        wh.time_batch_kernel(batch, reps=5, workspace=wsp, n_defl=nds, **kw)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "traffic", "copy_bytes_each_way": a.numel() * 8}), flush=True)
        return

    log(f"bench: {len(probs)} problems, warmup {args.warmup}, steps {args.steps}")
    for i in range(args.warmup):
        us, infos = wh.solve_batched(batch, workspace=wsp, n_defl=nds, **kw)
        log(f"warmup {i}: {infos[0]['ms']:.1f} ms")
    torch.cuda.synchronize()
    step_s = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        us, infos = wh.solve_batched(batch, workspace=wsp, n_defl=nds, **kw)
        step_s.append(time.perf_counter() - ts)      # each batched solve ends in a host read-back
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    # wave-step throughput of the batch: interior points x N_t of every wave solve (FP32 and FP64)
    psteps = sum((i["wave_solves"] + i["wave_solves_f32"]) * i["nt"] * (q.n - 1) ** 2 for i, q in zip(infos, probs))
    value = psteps / (ms / 1e3) / 1e9
    statuses = {str(k): sum(1 for i in infos if i["status"] == k) for k in sorted(set(i["status"] for i in infos))}
    log(f"timed: {ms:.1f} ms per batch, {value:.1f} Gpts/s, statuses {statuses}")
    hres = [wh.helmholtz_residual(u, f, q.omega) for u, f, q in zip(us, fs, probs)]

    # roofline of the dominant kernel: the batched FP32 work kernel (K register-tiled leapfrog
    # steps + FP64 filter sum on every tile of every problem), every problem in its stepping
    # phase, timed with HIP events on the library's stream (torch's current stream)
    launch_us, pts = wh.time_batch_kernel(batch, reps=20, workspace=wsp, n_defl=nds, **kw)
    bytes_launch = B_FUSED_F32 * pts
    achieved = bytes_launch / (launch_us * 1e-6) / 1e9
    stream_eq = B_PER_PT_STEP_F32 * pts * K / (launch_us * 1e-6) / 1e9
    log(f"batch kernel: {launch_us:.1f} us per launch, {pts} points x {K} steps, {achieved:.0f} GB/s fused-form")
    copy_gbs = _copy_gbs(torch)
    traffic = _traffic_lookup()

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": f"{len(probs)} batched 2D Dirichlet solves, {args.per_size} each on 128^2, 256^2, "
                               "512^2, 1024^2, omega~U(10,80) off resonance, source omega^2 exp(-omega^2 r^2) at "
                               "seeded centres (seed 4), DCG with the floor(1.5 omega) sine modes nearest omega^2, "
                               "FP32 stepping / FP64 filter+Krylov, graph-replayed rounds, true residual 1e-8",
                   "problems": len(probs), "solver": "dcg", "precision": "mixed", "tol": 1e-8, "k_fuse": K,
                   "tile": f"{infos[0]['k_waves']} row-marching strips of {64 - 2 * K} columns x "
                           f"{infos[0]['k_rows']} rows", "n_defl_rule": "floor(1.5 omega)"},
        "time_to_tol_ms_per_batch": round(ms, 3),
        "time_to_tol_ms_per_solve": round(ms / len(probs), 4),
        "ms_per_step_min_median": [round(min(step_s) * 1e3, 3), round(sorted(step_s)[len(step_s) // 2] * 1e3, 3)],
        "solve": {"status_counts": statuses, "iters": int(sum(i["iters"] for i in infos)),
                  "wave_solves_f32": int(sum(i["wave_solves_f32"] for i in infos)),
                  "wave_solves_f64": int(sum(i["wave_solves"] for i in infos)),
                  "point_steps": int(psteps),
                  "max_true_rel_res": max(i["true_rel_res"] for i in infos),
                  "max_helmholtz_rel_res": max(hres), "median_helmholtz_rel_res": float(np.median(hres))},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": f"k_batch_tile<float,{K},false,1> (the solver's FP32 row-marching work kernel under its "
                               "measurement tag: K leapfrog steps + FP64 filter sum per launch on every tile)",
                     "bytes_per_point_per_launch": B_FUSED_F32, "points_per_launch": pts, "k_fuse": K,
                     "bytes_per_launch": bytes_launch, "launch_us": round(launch_us, 3),
                     "streaming_equivalent_gbs": round(stream_eq, 1),
                     "streaming_equivalent_bytes_per_pt_step": B_PER_PT_STEP_F32,
                     "hbm_gbs_from_traffic": None if traffic is None else round(traffic / (launch_us * 1e-6) / 1e9, 1),
                     "copy_gbs": round(copy_gbs, 1)},
    }
    # same 256 problems in the other forms, once each (their solutions kept on the host for the
    # oracle comparison of the CPU leg)
    others = {}
    if not args.no_f64:
        for solver in ("dcg", "cg"):
            dk = dict(solver=solver, tol=1e-8, max_iters=100000, precision="f64")
            for f, q in zip(fs[:: args.per_size], probs[:: args.per_size]):     # autotune per size first
                wh.solve(f, q.omega, **{**dk, "max_iters": 2},
                         **({"defl": wh.sine_deflation(2, q.n, q.omega, 4)} if solver == "dcg" else {}))
            defl = [wh.sine_deflation(2, q.n, q.omega, nd) for q, nd in zip(probs, nds)] if solver == "dcg" else None
            res, dt = _timed(torch, lambda: [wh.solve(f, q.omega, **dk, **({"defl": defl[j]} if defl else {}))
                                            for j, (f, q) in enumerate(zip(fs, probs))])
            others[f"single_f64_{solver}"] = [u.cpu().numpy() for u, _ in res]
            line[f"single_f64_{solver}"] = {
                "seconds": round(dt, 3), "iters": int(sum(i["iters"] for _, i in res)),
                "status_counts": {str(k): sum(1 for _, i in res if i["status"] == k)
                                  for k in sorted(set(i["status"] for _, i in res))},
                "speedup_of_batched_mixed_dcg": round(dt / (ms / 1e3), 2)}
    if not args.no_cg:
        kcg = dict(kw, solver="cg")
        (ucg, icg), dt = _timed(torch, lambda: wh.solve_batched(batch, **kcg))
        others["batched_mixed_cg"] = [u.cpu().numpy() for u in ucg]
        blk = {"seconds": round(dt, 3), "iters": int(sum(i["iters"] for i in icg)),
               "status_counts": {str(k): sum(1 for i in icg if i["status"] == k) for k in sorted(set(i["status"] for i in icg))},
               "max_true_rel_res": max(i["true_rel_res"] for i in icg),
               "not_converged": [{"n": q.n, "omega": round(q.omega, 4), "status": i["status"], "iters": i["iters"],
                                  "outer": i["outer"], "true_rel_res": i["true_rel_res"]}
                                 for i, q in zip(icg, probs) if i["status"] != 0]}
        if "single_f64_cg" in line:
            blk["speedup_vs_single_f64_cg"] = round(line["single_f64_cg"]["seconds"] / dt, 3)
        line["batched_mixed_cg"] = blk
    # the previous single-solve line (1024^2 mixed DCG), kept as an extra key
    line["cfg2_single_solve"], cfg2_u = _cfg2_brief(np, torch, wh, wl)
    # the stepping kernels of the largest single solve (256^3, variable c), kept as an extra key;
    # its solves take minutes and run under --workload cfg3
    p3 = wl.config3()
    line["cfg3_stepping"] = {"workload": "3D 256^3, variable c (seed 3), omega=40: one blocked launch",
                             **_cfg3_step_kernels(torch, wh, wl, p3, torch.from_numpy(p3.c2).cuda())}
    del p3
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_cfg4(probs, [u.cpu().numpy() for u in us], infos, others,
                                                 (wl.config2(), cfg2_u))
    print(json.dumps(line), flush=True)


def _copy_gbs(torch):
    """The box's attainable HBM rate: a plain 1 GiB device-to-device copy (read + write)."""
    ca = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        cb.copy_(ca)
    e1.record()
    torch.cuda.synchronize()
    return 2 * ca.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9


def _batch_src_sha1():
    """sha1 over the code of the batched work kernel's sources (driver, state header, row-marching
    pipeline), with whole-line // comments and blank lines left out, so that a change of wording
    alone keeps the counters valid."""
    import hashlib
    h = hashlib.sha1()
    for f in ("wh_batched.hip", "wh_batched.h", "wh_march2d.h"):
        with open(os.path.join(ROOT, "paper_2606_31842_amd", "csrc", f)) as fh:
            for line in fh:
                t = line.strip()
                if t and not t.startswith("//"):
                    h.update(line.rstrip().encode() + b"\n")
    return h.hexdigest()


def _traffic_lookup():
    """HBM bytes per launch of the tagged batch kernel from the two counter passes summarised in
    profiles/hbm_traffic_batch_tile_cfg4.md, or None when the kernel sources have changed since."""
    if not BATCH_TRAFFIC["kib"] or _batch_src_sha1() != BATCH_TRAFFIC["src_sha1"]:
        return None
    fk, wk = BATCH_TRAFFIC["kib"]
    return round(1024 * (fk * BATCH_TRAFFIC["fetch_scale"] + wk * BATCH_TRAFFIC["write_scale"]))


def _cfg2_brief(np, torch, wh, wl):
    p = wl.config2()
    f = torch.from_numpy(p.f).cuda()
    kw = dict(solver="dcg", defl=wh.sine_deflation(2, p.n, p.omega, 32), precision="mixed", tol=1e-8,
              max_iters=50000, k_fuse=8, k_shape=1)
    wh.solve(f, p.omega, **kw)
    (u, info), dt = _timed(torch, lambda: wh.solve(f, p.omega, **kw))
    steps = (info["wave_solves"] + info["wave_solves_f32"]) * info["nt"]
    return {"workload": "2D 1024^2, c=1, omega=100.3, mixed DCG with 32 sine modes, tol 1e-8",
            "time_to_tol_ms": round(dt * 1e3, 2), "gpts": round((p.n - 1) ** 2 * steps / dt / 1e9, 1),
            "iters": info["iters"], "true_rel_res": info["true_rel_res"],
            "helmholtz_rel_res": wh.helmholtz_residual(u, f, p.omega)}, u.cpu().numpy()


def _dst_job(args):
    from oracle import discretization as disc
    n, omega, f = args
    return disc.direct_solve_dst(2, n, omega, f)


def cpu_baseline_cfg4(probs, sols, infos, others=None, single=None, budget_s=20.0):
    """The oracle on the host for the batch: (1) its FP64 WaveHoltz CG (the iteration the GPU
    runs, step by step in scipy) on a bounded sample -- the 128^2 problems over a spawn pool of
    every visible core, until about budget_s -- as wave-step Gpts/s; (2) its direct solve of every
    problem's discrete Helmholtz system (sine transform, exact for c = 1), timed, and the
    element-wise error of each GPU solution against it: the batch's, those of the comparison
    runs on the same problems (`others`: name -> solutions), and that of the single 1024^2
    solve (`single`: (problem, solution))."""
    import multiprocessing as mp
    import numpy as np
    cores = len(os.sched_getaffinity(0))
    ctx = mp.get_context("spawn")
    small = [q for q in probs if q.n == min(q.n for q in probs)]
    with ctx.Pool(cores) as pool:
        t0 = time.perf_counter()
        res = []
        for k in range(0, len(small), cores):
            res += pool.map(_oracle_cg_job, [(2, q.n, q.omega, q.f, 1e-8) for q in small[k:k + cores]])
            if time.perf_counter() - t0 > budget_s:
                break
        wall = time.perf_counter() - t0
        done = small[:len(res)]
        psteps = sum((it + 1) * nt * (q.n - 1) ** 2 for (it, nt, _), q in zip(res, done))
        t1 = time.perf_counter()
        exact = pool.map(_dst_job, [(q.n, q.omega, q.f) for q in probs])
        t_dst = time.perf_counter() - t1
    def err(u, U):
        return float(np.abs(u - U).max() / np.abs(U).max())
    errs = [err(u, U) for u, U in zip(sols, exact)]
    other_errs = {}
    for k, v in (others or {}).items():
        e = [err(u, U) for u, U in zip(v, exact)]
        j = int(np.argmax(e))
        other_errs[k] = {"max": e[j], "median": float(np.median(e)),
                         "at_max": {"n": probs[j].n, "omega": round(probs[j].omega, 4)}}
    if single is not None:
        q, u = single
        other_errs["cfg2_single_solve"] = {"max": err(u, _dst_job((q.n, q.omega, q.f)))}
    by_n = {}
    for q, e in zip(probs, errs):
        by_n.setdefault(q.n, []).append(e)
    return {"value": round(psteps / wall / 1e9, 4), "unit": "Gpts/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle FP64 WaveHoltz CG (scipy CSR leapfrog) to 1e-8 on {len(res)} of the {len(small)} "
                      f"problems of size {small[0].n}, a spawn pool of {cores} processes, {wall:.1f} s; host "
                      f"{cpu_model()}",
            "sample_wall_s": round(wall, 2), "sample_iters": int(sum(r[0] for r in res)),
            "direct_dst_all_s": round(t_dst, 2),
            "error_vs_oracle_max_elementwise": max(errs),
            "error_vs_oracle_by_size_max": {str(k): max(v) for k, v in sorted(by_n.items())},
            "error_vs_oracle_each": [float(f"{e:.3g}") for e in errs],
            "error_vs_oracle_max_other_runs": other_errs,
            "error_note": "max_i |u_i - U_i| / max|U| per solution against the oracle's direct solve (sine "
                          "transform) of the same discrete Helmholtz system; for the other runs the maximum "
                          "and median over their solutions and the problem at the maximum"}



def _timed(torch, fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t


def run_cfg1(args, np, torch, wh, wl):
    """2D 64^2, c = 1, omega = 20.5, FP64 CG to 1e-10."""
    p = wl.config1()
    f = torch.from_numpy(p.f).cuda()
    kw = dict(solver="cg", precision="f64", tol=1e-10)
    wh.solve(f, p.omega, **kw)
    (u, info), dt = _timed(torch, lambda: wh.solve(f, p.omega, **kw))
    steps = (info["wave_solves"] + info["wave_solves_f32"]) * info["nt"]
    out = {"workload": "cfg1 2D 64^2 FP64 CG tol 1e-10", "time_to_tol_ms": dt * 1e3,
           "gpts": (p.n - 1) ** 2 * steps / dt / 1e9, "iters": info["iters"], "nt": info["nt"],
           "true_rel_res": info["true_rel_res"], "helmholtz_rel_res": wh.helmholtz_residual(u, f, p.omega)}
    if not args.no_cpu:
        it, nt, sec = oracle_cg_solve(2, p.n, p.omega, p.f, 1e-10)
        out["cpu_baseline"] = {"kind": "oracle", "cores": 1, "oracle_cg_seconds": round(sec, 3), "oracle_cg_iters": it,
                               "oracle_gpts": (p.n - 1) ** 2 * nt * (it + 1) / sec / 1e9,
                               "direct_splu": direct_splu(2, p.n, p.omega, p.f), "host": cpu_model()}
    return out


def _cfg3_step_kernels(torch, wh, wl, p, c2):
    """Per-launch time of the autotuned 3D blocked stepping kernel on the 256^3 variable-c grid,
    FP32 and FP64 (HIP events inside the library, 20 launches)."""
    pts = (p.n - 1) ** 3
    out = {}
    v = torch.from_numpy(wl.random_nodal(3, p.n, 1)).cuda()
    for prec in ("mixed", "f64"):
        ms, sh = wh.time_step_kernel(v, p.omega, c2=c2, precision=prec, reps=20, shape=True)
        us = ms * 1e3
        k = max(1, sh["k"])
        # streaming-form algorithmic bytes per point-step (variable c): FP32 state 4+4 in, 4 out,
        # kap 4, V 16; FP64: 8+8 in, 8 out, kap 8, V 16
        bpp = 32.0 if prec == "mixed" else 48.0
        out[f"step_kernel_{prec}"] = {"us_per_launch": us, "k_fuse": k, "rows": sh["rows"], "waves": sh["waves"],
                                      "us_per_step": us / k, "gpts": pts * k / us / 1e3, "bytes_per_pt_step": bpp,
                                      "achieved_gbs": bpp * pts * k / (us * 1e-6) / 1e9}
    return out


def run_cfg3(args, np, torch, wh, wl):
    """3D 256^3, seeded variable c, omega = 40: GMRES(40) (mixed and FP64, capped) and CG (FP64 and mixed) to
    a true residual of 1e-8, with the Helmholtz residual as the accuracy check at this size."""
    p = wl.config3()
    f = torch.from_numpy(p.f).cuda()
    c2 = torch.from_numpy(p.c2).cuda()
    pts = (p.n - 1) ** 3
    out = {"workload": "cfg3 3D 256^3 variable c omega=40 mixed tol 1e-8"}
    out.update(_cfg3_step_kernels(torch, wh, wl, p, c2))
    if args.probe_traffic:
        return out
    # GMRES(40) as the workload states it (capped: it stalls near resonance); CG to the
    # tolerance in both precisions
    # FP64 GMRES(40) beside the mixed one separates restart stagnation from the FP32 operator
    runs = [("gmres", "mixed", args.max_iters or 2000), ("gmres", "f64", args.max_iters or 2000),
            ("cg", "f64", 20000), ("cg", "mixed", 20000)]
    for solver, prec, cap in runs:
        wh.solve(f, p.omega, c2=c2, solver=solver, precision=prec, tol=1e-8, max_iters=2, restart=40)
        (u, info), dt = _timed(torch, lambda: wh.solve(f, p.omega, c2=c2, solver=solver, precision=prec,
                                                      tol=1e-8, max_iters=cap, restart=40))
        log(f"cfg3 {solver} {prec}: {dt:.1f} s, status {info['status']}, iters {info['iters']}")
        out[f"{solver}_{prec}"] = {"seconds": dt, "status": info["status"], "iters": info["iters"], "cap": cap,
                                   "true_rel_res": info["true_rel_res"], "helmholtz_rel_res":
                                   wh.helmholtz_residual(u, f, p.omega, c2), "nt": info["nt"],
                                   "wave_solves_f32": info["wave_solves_f32"], "wave_solves_f64": info["wave_solves"]}
    if not args.no_cpu:
        from oracle import discretization as disc, timeparams as tpm, wavesolve as ws
        with _one_thread():
            L = disc.laplacian(3, p.n, p.c2)
            tp = tpm.time_parameters(p.omega, 1.0 / p.n, float(np.sqrt(p.c2.max())))
            v = disc.to_interior(p.f)
            t0 = time.perf_counter()
            for _ in range(3):
                v = ws.apply_S(L, v, tp)
            per = (time.perf_counter() - t0) / 3
        cb = {"kind": "oracle", "cores": 1, "host": cpu_model(), "s_per_wave_solve": round(per, 2), "nt": tp.nt,
              "oracle_gpts": pts * tp.nt / per / 1e9,
              "sample": "3 FP64 wave solves of the variable-c 256^3 operator (scipy CSR, one thread)"}
        for key in ("gmres_mixed", "gmres_f64", "cg_f64", "cg_mixed"):
            nws = out[key]["wave_solves_f32"] + out[key]["wave_solves_f64"]
            cb[f"{key}_extrapolated_seconds"] = round(per * nws, 1)
        out["cpu_baseline"] = cb
    return out


def run_cfg5(args, np, torch, wh, wl):
    """Adjoint gradient on 513^2 with 16 sources and 4 x 128 receivers; one GPU central
    difference of J in a random direction as a check."""
    wk = wl.config5()
    c2 = torch.from_numpy(wk.c2).cuda()
    srcs = [torch.from_numpy(f).cuda() for f in wk.sources]
    rec = torch.from_numpy(wk.rec_idx)
    # data from the reference c2 with the library's own solves
    c2r = torch.from_numpy(wk.c2_ref).cuda()
    d = torch.stack([wh.solve(f, wk.omega, c2=c2r, tol=1e-12, max_iters=20000, c_max=wk.c_max)[0].reshape(-1)[rec.cuda()]
                     for f in srcs])
    kw = dict(tol=1e-10, c_max=wk.c_max, max_iters=20000)
    (J, g, info), dt = _timed(torch, lambda: wh.adjoint_grad(c2, srcs, rec, d, wk.omega, ckpt_every=16, **kw))
    # central differences of J (misfit only, FP64, tol 1e-12) in each of the random directions
    eps = 1e-6
    kw12 = dict(kw, tol=1e-12)
    gaps, fds, ans = [], [], []
    t0 = time.perf_counter()
    for k, dirk in enumerate(wk.directions[:args.fd_directions]):
        delta = torch.from_numpy(dirk).cuda()
        Jp = wh.adjoint_grad(c2 + eps * delta, srcs, rec, d, wk.omega, need_grad=False, **kw12)[0]
        Jm = wh.adjoint_grad(c2 - eps * delta, srcs, rec, d, wk.omega, need_grad=False, **kw12)[0]
        fd = (Jp - Jm) / (2 * eps)
        an = float((g * delta).sum())
        fds.append(fd)
        ans.append(an)
        gaps.append(abs(fd - an) / abs(an))
        log(f"direction {k}: FD {fd:.9e} adjoint {an:.9e} rel gap {gaps[-1]:.2e}")
    t_fd = time.perf_counter() - t0
    return {"workload": "cfg5 adjoint 513^2, 16 sources, 512 receivers, omega=30, ckpt 16",
            "seconds": dt, "J": J, "iters": info["iters"], "nt": info["nt"], "wave_solves": info["wave_solves"],
            "fd_directions": len(gaps), "fd_eps": eps, "fd_tol": 1e-12, "fd_seconds": t_fd,
            "fd_rel_gap_max": max(gaps) if gaps else None,
            "fd_rel_gap_median": float(np.median(gaps)) if gaps else None,
            "fd_directional": fds, "adjoint_directional": ans}


def _explicit_modes(np, torch, wh, n, omega, nd, form):
    """The nd sine modes nearest resonance given explicitly instead of by mode numbers, each
    degenerate pair (a, b), (b, a) rotated by 45 degrees (still eigenvectors, rank 2 on the
    grid): as dense nodal columns, or as their separable factors."""
    modes, lam2 = wh.select_sine_modes(2, n, omega, nd)
    x = np.arange(n + 1) / n
    s1 = lambda k: np.sqrt(2.0 / n) * np.sin(np.pi * k * x)
    vecs = [np.outer(s1(b), s1(a)) for a, b in modes]          # [y][x]
    pairs = {(int(a), int(b)): i for i, (a, b) in enumerate(modes)}
    for (a, b), i in pairs.items():
        j = pairs.get((b, a), -1)
        if j > i:
            u, v = vecs[i], vecs[j]
            vecs[i], vecs[j] = (u + v) / np.sqrt(2.0), (u - v) / np.sqrt(2.0)
    V = np.stack(vecs)
    if form == "dense":
        Vt = torch.from_numpy(V.reshape(nd, -1)).cuda()
        return wh.Deflation(wh.WH_DEFL_DENSE_EXACT, V=Vt, lambda2=lam2)
    from compress_modes import compress_modes
    fx, fy, tm, ranks = compress_modes(V, tol=1e-12)
    return wh.factored_deflation(fx, fy, tm, lam2)


def run_solvers(args, np, torch, wh, wl):
    """The config-2 problem (2D 1024^2, omega = 100.3) by every solver of the library, true
    residual 1e-8: CG, DCG with N_D sine modes, Algorithm 2 (DEVD) around CG, GMRES(40),
    BiCGStab and both augmented with the modes (Algorithms 4, 5) in mixed precision; DEVD around FPI with deflated iterates
    in FP64.  Accuracy as the library's Helmholtz residual."""
    p = wl.config2()
    n = p.n
    f = torch.from_numpy(p.f).cuda()
    cap = args.max_iters or 6000
    runs = [("cg", 0, {}), ("dcg", 8, {}), ("dcg", 32, {}), ("dcg", 64, {}),
            ("cg", 32, {"devd": 1}), ("fpi", 32, {"devd": 2}), ("gmres", 0, {}), ("gmres", 32, {}),
            ("bicgstab", 0, {}), ("bicgstab", 32, {}), ("gmres", 32, {"form": "dense"}),
            ("gmres", 32, {"form": "factored"})]
    out = {"workload": "config-2 problem (2D 1024^2, c = 1, omega = 100.3) by every solver, tol 1e-8",
           "max_iters": cap}
    only = [r for r in args.runs.split(",") if r]
    for solver, nd, extra in runs:
        name = ("devd_" if extra.get("devd") else "") + solver + (f"_nd{nd}" if nd else "")
        if solver in ("gmres", "bicgstab") and nd:
            name = f"a{solver}_nd{nd}" + (f"_{extra['form']}" if "form" in extra else "")
        if only and name not in only:
            continue
        # the fixed-point iteration runs in FP64 only
        form = extra.pop("form", "sine") if "form" in extra else "sine"
        kw = dict(solver=solver, precision="f64" if solver == "fpi" else "mixed", tol=1e-8, max_iters=cap,
                  restart=40, **extra)
        if nd:
            kw["defl"] = wh.sine_deflation(2, n, p.omega, nd) if form == "sine" else \
                _explicit_modes(np, torch, wh, n, p.omega, nd, form)
        wh.solve(f, p.omega, **{**kw, "max_iters": 2})   # autotune and warm up outside the timing
        (u, info), dt = _timed(torch, lambda: wh.solve(f, p.omega, **kw))
        out[name] = {"seconds": dt, "precision": kw["precision"], "status": info["status"], "iters": info["iters"],
                     "wave_solves_f32": info["wave_solves_f32"], "wave_solves_f64": info["wave_solves"],
                     "true_rel_res": info["true_rel_res"],
                     "helmholtz_rel_res": wh.helmholtz_residual(u, f, p.omega)}
        log(name, out[name])
    return out


def run_ndsweep(args, np, torch, wh, wl):
    """Iterations against omega for the two deflation-size rules of the paper's frequency
    study (Section 4.2): N_D = floor(3 omega / 2) and floor(omega^2 / 10).  Per omega: CG
    without deflation, DCG, Algorithm 2 around CG (CG with f_d) and around the fixed-point
    iteration (WHI with f_d), FP64, true residual 1e-8, on the unit square with n from the
    PPW rule (second order, eps = 1e-3)."""
    if ":" in args.omegas:
        a, b = (int(t) for t in args.omegas.split(":"))
        omegas = list(range(a, b + 1))
    else:
        omegas = [float(t) for t in args.omegas.split(",") if t]
    cap = args.max_iters or 5000
    rows = []
    for om in omegas:
        q = wl.ndsweep_problem(om)
        f = torch.from_numpy(q.f).cuda()
        kw = dict(precision="f64", tol=1e-8, max_iters=cap)
        wh.solve(f, q.omega, solver="cg", **{**kw, "max_iters": 2})   # autotune outside the timing
        row = {"omega": om, "n": q.n}
        (u, i), dt = _timed(torch, lambda: wh.solve(f, q.omega, solver="cg", **kw))
        row["cg"] = {"iters": i["iters"], "status": i["status"], "seconds": dt}
        for rule, nd in (("lin", int(math.floor(1.5 * om))), ("quad", int(math.floor(om * om / 10.0)))):
            d = wh.sine_deflation(2, q.n, q.omega, nd)
            row[f"nd_{rule}"] = nd
            for name, extra in (("dcg", dict(solver="dcg")), ("devd_cg", dict(solver="cg", devd=1)),
                                ("devd_whi", dict(solver="fpi", devd=1))):
                (u, i), dt = _timed(torch, lambda: wh.solve(f, q.omega, defl=d, **kw, **extra))
                row[f"{name}_{rule}"] = {"iters": i["iters"], "status": i["status"], "seconds": dt}
        log(f"omega {om}: n {q.n} cg {row['cg']['iters']} | lin N_D {row['nd_lin']}: dcg "
            f"{row['dcg_lin']['iters']} devd_cg {row['devd_cg_lin']['iters']} whi {row['devd_whi_lin']['iters']}"
            f" | quad N_D {row['nd_quad']}: dcg {row['dcg_quad']['iters']} devd_cg "
            f"{row['devd_cg_quad']['iters']} whi {row['devd_whi_quad']['iters']}")
        rows.append(row)
    return {"workload": "deflation-size sweep (unit square, c = 1, PPW grid eps 1e-3, FP64, tol 1e-8)",
            "rows": rows}


def run_order4(args, np, torch, wh, wl):
    """Fourth-order differences (c = 1), 2D: the stepping rate of the blocked launches (K = 4,
    the row-marching pipeline with the radius-2 stencil) against one step per launch, FP64 and
    FP32, on 2048^2 and 4096^2 grids; and a 1024^2 DCG solve (16 sine modes, tol 1e-8) timed
    both ways.  Fused-form bytes of a K-step launch per interior point: FP64 48 (state pair in
    and out, V read and written), FP32 32."""
    rows = []
    for n in (2048, 4096):
        v = torch.zeros((n + 1, n + 1), dtype=torch.float64, device="cuda")
        for prec in ("f64", "mixed"):
            for k in (1, 4):
                ms, sh = wh.time_step_kernel(v, 0.3 * n, precision=prec, reps=30, shape=True, order=4, k_fuse=k)
                K = max(sh["k"], 1)
                pts = (n - 1) ** 2
                row = {"n": n, "precision": prec, "k": sh["k"], "us_per_launch": round(1e3 * ms, 2),
                       "gpts_steps_per_s": round(pts * K / ms / 1e6, 1)}
                if K > 1:
                    bpp = 48 if prec == "f64" else 32
                    gbs = bpp * pts / (ms * 1e-3) / 1e9
                    row["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                                       "frac": round(gbs / 8000.0, 3)}
                log(f"order 4 stepping n={n} {prec} K={sh['k']}: {row['us_per_launch']} us per launch, "
                    f"{row['gpts_steps_per_s']} G point-steps/s")
                rows.append(row)
        del v
    n = 1024
    f = torch.from_numpy(wl.gaussian(2, n, (0.41, 0.57), 0.02)).cuda()
    om = 0.25 * n
    d = wh.sine_deflation(2, n, om, 16, order=4)
    solves = []
    for prec in ("f64", "mixed"):
        for k in (1, 4):
            kw = dict(solver="dcg", defl=d, tol=1e-8, max_iters=5000, order=4, precision=prec, k_fuse=k)
            wh.solve(f, om, **{**kw, "max_iters": 2})
            (u, i), dt = _timed(torch, lambda: wh.solve(f, om, **kw))
            solves.append({"precision": prec, "k": i["k_fuse"], "status": i["status"], "iters": i["iters"],
                           "seconds": round(dt, 3), "true_rel_res": i["true_rel_res"]})
            log(f"order 4 DCG n={n} {prec} K={i['k_fuse']}: {i['iters']} iterations, {dt:.3f} s")
    return {"workload": "fourth-order 2D stepping (c = 1) and a 1024^2 DCG solve (omega = 256, 16 sine modes)",
            "stepping": rows, "solves": solves}


EXTRA = {"cfg1": run_cfg1, "cfg2": run_cfg2, "solvers": run_solvers, "ndsweep": run_ndsweep, "cfg3": run_cfg3, "cfg5": run_cfg5,
         "order4": run_order4}


if __name__ == "__main__":
    main()
