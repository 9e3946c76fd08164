"""GPU parity of wh_solve_batched: every problem of a mixed-size, mixed-frequency
batch against the oracle's direct Helmholtz solve, and against wh_solve."""
import numpy as np
import pytest

import workloads as wl
from oracle import discretization as disc
from _gpu import cuda, host, direct, assert_close, relmx

pytestmark = pytest.mark.gpu


def _batch(sizes=(24, 40, 64, 101), per=2, seed=9, omega=(8.0, 30.0)):
    rng = np.random.default_rng(seed)
    probs = []
    for n in sizes:
        for _ in range(per):
            while True:
                om = float(rng.uniform(*omega))
                if wl.gap_ok(n, om, 0.05):
                    break
            x0 = rng.uniform(0.2, 0.8, 2)
            probs.append((n, om, wl.gaussian(2, n, x0, 1.0 / om, amplitude=om * om)))
    return probs


@pytest.mark.parametrize("precision,k_fuse", [("f64", 4), ("mixed", 4), ("f64", 8), ("mixed", 2)])
def test_batched_matches_direct_and_single(precision, k_fuse):
    print(f"case batched {precision} K={k_fuse}", flush=True)
    import paper_2606_31842_amd as wh
    probs = _batch()
    tol = 1e-12 if precision == "f64" else 1e-9
    us, infos = wh.solve_batched([(cuda(f), om) for (n, om, f) in probs], precision=precision, tol=tol,
                                 k_fuse=k_fuse, max_iters=20000)
    for (n, om, f), u, info in zip(probs, us, infos):
        U = disc.direct_solve_dst(2, n, om, f)
        print(f"n={n} omega={om:.3f} status={info['status']} iters={info['iters']} outer={info['outer']} "
              f"true={info['true_rel_res']:.2e}", flush=True)
        assert info["status"] == 0
        assert info["true_rel_res"] <= (1.5 * tol if precision == "f64" else tol)
        assert_close(host(u), U, 1e-10 if precision == "f64" else 2e-5, "vs direct")
        if precision == "f64":
            # same algorithm as the single solve: same iteration count, same iterate
            us1, i1 = wh.solve(cuda(f), om, solver="cg", tol=tol, max_iters=20000)
            assert abs(i1["iters"] - info["iters"]) <= 1
            assert_close(host(u), host(us1), 1e-10, "vs single solve")


def test_batched_variable_c():
    import paper_2606_31842_amd as wh
    rng = np.random.default_rng(4)
    probs = []
    for n, om in ((32, 11.3), (48, 17.9), (30, 9.1)):
        c2 = wl.config5_c2(n, rng)
        probs.append((n, om, wl.gaussian(2, n, rng.uniform(.3, .7, 2), 0.1), c2))
    us, infos = wh.solve_batched([(cuda(f), om, cuda(c2)) for (n, om, f, c2) in probs], precision="f64",
                                 tol=1e-11, c_max=float(np.sqrt(1.2)), max_iters=20000)
    for (n, om, f, c2), u, info in zip(probs, us, infos):
        U = direct(2, n, om, f, c2)
        assert info["status"] == 0
        assert relmx(host(u), U) < 1e-8


def test_batched_rejects_bad_input():
    import paper_2606_31842_amd as wh
    f = cuda(wl.gaussian(2, 16, (0.5, 0.5), 0.1))
    with pytest.raises(wh.WaveHoltzError):
        wh.solve_batched([(f, 5.0)], solver="gmres")
    with pytest.raises(wh.WaveHoltzError):
        wh.solve_batched([(f, 5.0, cuda(np.ones((17, 17))))])   # variable c without c_max


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_batched_dcg_matches_direct_and_single(precision):
    """Deflated batches (sine modes nearest omega^2): the start x_0 = W (W^T A W)^{-1} W^T b
    of Algorithm 3, then CG; one problem of the batch runs undeflated."""
    print(f"case batched dcg {precision}", flush=True)
    import paper_2606_31842_amd as wh
    probs = _batch(seed=21, omega=(12.0, 40.0))
    nds = [8 if i % 4 else 0 for i in range(len(probs))] if precision == "mixed" else [8] * len(probs)
    tol = 1e-9
    us, infos = wh.solve_batched([(cuda(f), om) for (n, om, f) in probs], precision=precision, tol=tol,
                                 solver="dcg", n_defl=nds, k_fuse=4, max_iters=20000)
    for (n, om, f), nd, u, info in zip(probs, nds, us, infos):
        U = disc.direct_solve_dst(2, n, om, f)
        e = relmx(host(u), U)
        print(f"n={n} omega={om:.3f} nd={nd} status={info['status']} iters={info['iters']} "
              f"true={info['true_rel_res']:.2e} err={e:.2e}", flush=True)
        assert info["status"] == 0
        assert info["true_rel_res"] <= (1.5 * tol if precision == "f64" else tol)
        assert e < (1e-6 if precision == "f64" else 2e-5)
        if precision == "f64":
            # the single solve with the same deflation set: same iteration count, same iterate
            u1, i1 = wh.solve(cuda(f), om, solver="dcg", defl=wh.sine_deflation(2, n, om, nd), tol=tol,
                              max_iters=20000)
            assert abs(i1["iters"] - info["iters"]) <= 2, (i1["iters"], info["iters"])
            assert relmx(host(u), host(u1)) < 1e-7


def test_batched_dcg_start_is_solution():
    """f inside the deflation space: the deflated start is the solution; no CG iteration."""
    import paper_2606_31842_amd as wh
    n, om = 48, 17.3
    modes, lam2 = wh.select_sine_modes(2, n, om, 4)
    x = np.arange(n + 1) / n
    f = sum((k + 1.0) * np.outer(np.sin(np.pi * b * x), np.sin(np.pi * a * x)) for k, (a, b) in enumerate(modes))
    us, infos = wh.solve_batched([(cuda(f), om)], solver="dcg", n_defl=4, tol=1e-10, precision="f64")
    U = disc.direct_solve_dst(2, n, om, f)
    assert infos[0]["status"] == 0 and infos[0]["iters"] == 0
    assert infos[0]["true_rel_res"] < 1e-10
    assert relmx(host(us[0]), U) < 1e-10


@pytest.mark.parametrize("solver,precision", [("cg", "f64"), ("cg", "mixed"), ("dcg", "mixed")])
def test_batched_zero_forcing_problem(solver, precision):
    """A problem with f = 0 inside a batch finishes at once with u = 0; the others solve."""
    import paper_2606_31842_amd as wh
    n1, n2, om = 48, 64, 17.3
    f1 = np.zeros((n1 + 1, n1 + 1))
    f2 = wl.gaussian(2, n2, (0.41, 0.57), 0.08)
    kw = dict(solver=solver, tol=1e-9, precision=precision, max_iters=5000)
    if solver == "dcg":
        kw["n_defl"] = [4, 4]
    us, infos = wh.solve_batched([(cuda(f1), om), (cuda(f2), om)], **kw)
    assert infos[0]["status"] == 0 and infos[0]["iters"] == 0
    assert np.abs(host(us[0])).max() == 0
    assert infos[1]["status"] == 0
    U = disc.direct_solve_dst(2, n2, om, f2)
    assert relmx(host(us[1]), U) < (1e-7 if precision == "f64" else 2e-5)


def test_batched_dcg_rejects_bad_input():
    import paper_2606_31842_amd as wh
    f = cuda(wl.gaussian(2, 16, (0.5, 0.5), 0.1))
    with pytest.raises(wh.WaveHoltzError):
        wh.solve_batched([(f, 5.0)], solver="cg", n_defl=2)          # deflation needs DCG
    with pytest.raises(wh.WaveHoltzError):
        wh.solve_batched([(f, 5.0, cuda(np.ones((17, 17))))], solver="dcg", n_defl=2,
                         c_max=1.0)                                   # sine modes need c == 1
    with pytest.raises(wh.WaveHoltzError):
        wh.solve_batched([(f, 5.0)], solver="dcg", n_defl=15 * 15 + 1)


def test_time_batch_kernel_reports_points_and_time():
    # the measurement helper of the batched FP32 work kernel: every problem in its stepping
    # phase; it returns the interior points one launch advances and a positive duration, and
    # leaves the solver usable (a solve afterwards still matches the direct solution)
    import torch
    import paper_2606_31842_amd as wh
    probs = [(wl.gaussian(2, n, (0.4, 0.6), 0.1), om) for n, om in ((40, 11.3), (64, 17.9), (33, 9.1))]
    batch = [(cuda(f), om) for f, om in probs]
    us, pts = wh.time_batch_kernel(batch, reps=5, k_fuse=4, solver="cg")
    assert pts == sum((f.shape[0] - 2) ** 2 for f, _ in probs)
    assert 0 < us < 1e5
    sols, infos = wh.solve_batched(batch, precision="mixed", tol=1e-9, k_fuse=4)
    for (f, om), u, info in zip(probs, sols, infos):
        n = f.shape[0] - 1
        U = direct(2, n, om, f)
        assert info["status"] == 0
        assert relmx(host(u), U) < 2e-5


def test_batched_mixed_cg_near_indefinite_problem_converges():
    # the 128^2 problem at omega = 76.0139 of the 256-problem workload has a degenerate pair of
    # modes whose A-eigenvalue is slightly negative (beta_h overshoots 1 just below omega with
    # 22 steps per period); the FP32 operator stalls on it, the problem falls back to FP64 and
    # restarts from zero as plain CG, and reaches the tolerance like the FP64 single solve
    import paper_2606_31842_amd as wh
    q = [p for p in wl.config4() if p.n == 128 and abs(p.omega - 76.0139) < 1e-3][0]
    other = [p for p in wl.config4() if p.n == 128][:2]
    probs = [q] + other
    sols, infos = wh.solve_batched([(cuda(p.f), p.omega) for p in probs], precision="mixed", solver="cg",
                                   tol=1e-8, k_fuse=8, max_iters=10000)
    for p, u, info in zip(probs, sols, infos):
        U = direct(2, p.n, p.omega, p.f)
        err = relmx(host(u), U)
        print(f"omega {p.omega:.4f}: status {info['status']} iters {info['iters']} fp64 solves "
              f"{info['wave_solves']} err {err:.2e}", flush=True)
        assert info["status"] == 0 and info["true_rel_res"] <= 1e-8
        assert err < 2e-5
    assert infos[0]["wave_solves"] > infos[0]["outer"] + 1    # it did run in FP64


@pytest.mark.parametrize("k_fuse", [8, 4, 2])
def test_batched_mixed_operator_needs_no_fp64_fallback(k_fuse):
    """Grids of two and more tile columns: the FP32 operator of the mixed batch must be accurate
    enough that no problem falls back to FP64 stepping (FP64 wave solves = the right-hand side
    plus one per residual replacement), and the mixed DCG takes about the iterations of the FP64
    one.  (A wrong FP32 operator still converges through the fallback; this catches it.)"""
    print(f"case batched mixed operator K={k_fuse}", flush=True)
    import paper_2606_31842_amd as wh
    probs = _batch(sizes=(130, 200, 260), per=2, seed=33, omega=(10.0, 30.0))
    batch = [(cuda(f), om) for (n, om, f) in probs]
    nds = [int(1.5 * om) for (n, om, f) in probs]   # every problem deflated: interleaved FP32 pairs
    kw = dict(solver="dcg", n_defl=nds, k_fuse=k_fuse, tol=1e-8, max_iters=20000)
    um, im = wh.solve_batched(batch, precision="mixed", **kw)
    u64, i64 = wh.solve_batched(batch, precision="f64", **kw)
    for (n, om, f), u, a, b in zip(probs, um, im, i64):
        U = disc.direct_solve_dst(2, n, om, f)
        e = relmx(host(u), U)
        print(f"n={n} omega={om:.3f} mixed iters={a['iters']} fp64 solves={a['wave_solves']} outer={a['outer']} "
              f"| f64 iters={b['iters']} err={e:.2e}", flush=True)
        assert a["status"] == 0 and e < 2e-5
        assert a["wave_solves"] == a["outer"] + 1, a
        assert a["iters"] <= 1.25 * b["iters"] + 5
