"""Edge cases of the solve entry point on the GPU, every solver: zero forcing, a zero
iteration budget, a tolerance met by the start, the smallest grid, ragged tile tails,
and a deflation set at its size limit."""
import numpy as np
import pytest

import workloads as wl
from oracle import discretization as disc, modes
from _gpu import cuda, host, relmx

pytestmark = pytest.mark.gpu

SOLVERS = [("fpi", {}), ("cg", {}), ("dcg", {"nd": 4}), ("gmres", {}), ("bicgstab", {}), ("gmres", {"nd": 4}),
           ("bicgstab", {"nd": 4}), ("cg", {"nd": 4, "devd": 1})]


def _kw(solver, extra, n, omega, dim=2):
    import paper_2606_31842_amd as wh
    kw = dict(solver=solver, restart=10)
    if "nd" in extra:
        kw["defl"] = wh.sine_deflation(dim, n, omega, extra["nd"])
    if "devd" in extra:
        kw["devd"] = extra["devd"]
    return kw


@pytest.mark.parametrize("solver,extra", SOLVERS)
@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_zero_forcing_gives_zero(solver, extra, precision):
    print(f"case zero forcing {solver} {extra} {precision}", flush=True)
    import paper_2606_31842_amd as wh
    if solver == "fpi" and precision == "mixed":
        pytest.skip("the fixed-point iteration runs in FP64 only")
    n, omega = 24, 7.3
    f = cuda(np.zeros((n + 1, n + 1)))
    u0 = cuda(wl.random_nodal(2, n, seed=3))
    u, info = wh.solve(f, omega, u0=u0, tol=1e-10, max_iters=500, precision=precision,
                       **_kw(solver, extra, n, omega))
    assert info["status"] == 0, info
    assert np.abs(host(u)).max() < 1e-8 * np.abs(host(u0)).max() + 1e-300


@pytest.mark.parametrize("solver,extra", SOLVERS)
def test_zero_iteration_budget_and_loose_tolerance(solver, extra):
    import paper_2606_31842_amd as wh
    n, omega = 32, 9.1
    f = cuda(wl.gaussian(2, n, (0.4, 0.6), 0.1))
    u, info = wh.solve(f, omega, tol=1e-10, max_iters=0, **_kw(solver, extra, n, omega))
    assert info["status"] == 1 and info["iters"] == 0 and np.all(np.isfinite(host(u)))
    # a tolerance of 2 is met by the zero start (||b - A 0|| / ||b|| = 1); the fixed-point
    # iteration measures its update ||Pi x - x||, which takes one application
    u, info = wh.solve(f, omega, tol=2.0, max_iters=100, **_kw(solver, extra, n, omega))
    assert info["status"] == 0 and info["iters"] == (1 if solver == "fpi" else 0)
    if "nd" not in extra and solver != "fpi":
        # with a deflation set the W part is solved exactly before any iteration (DCG start,
        # augmented methods, DEVD inflation)
        assert np.abs(host(u)).max() == 0


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 4), (2, 66), (2, 113)])
@pytest.mark.parametrize("solver", ["cg", "gmres", "bicgstab"])
def test_small_and_ragged_grids(dim, n, solver):
    """The smallest grid (one interior node per axis beyond the boundary ring of 3) and
    sizes that leave ragged tails in the 48-, 52- and 64-wide tiles."""
    print(f"case grid dim={dim} n={n} {solver}", flush=True)
    import paper_2606_31842_amd as wh
    omega = 2.1 if n == 4 else 11.7
    f = wl.gaussian(dim, n, (0.45, 0.55, 0.5)[:dim], 0.2)
    u, info = wh.solve(cuda(f), omega, solver=solver, tol=1e-11, max_iters=3000, restart=20)
    assert info["status"] == 0, info
    U = disc.to_nodal(disc.direct_solve(disc.laplacian(dim, n), omega, disc.to_interior(f)), dim, n)
    assert relmx(host(u), U) < 1e-8


def test_largest_deflation_set():
    """n_d = 256, the largest set: DCG with it, against the direct solve."""
    import paper_2606_31842_amd as wh
    n, omega = 96, 40.3
    f = wl.gaussian(2, n, (0.41, 0.57), 0.06)
    d = wh.sine_deflation(2, n, omega, 256)
    u, info = wh.solve(cuda(f), omega, solver="dcg", defl=d, tol=1e-10, max_iters=3000)
    assert info["status"] == 0
    U = disc.direct_solve_dst(2, n, omega, f)
    assert relmx(host(u), U) < 1e-8
    with pytest.raises(wh.WaveHoltzError):
        wh.solve(cuda(f), omega, solver="dcg", defl=wh.sine_deflation(2, n, omega, 257))
