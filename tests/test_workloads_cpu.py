"""CPU checks of the seeded workload recipes that size grids from the paper's rules."""
import math

import numpy as np

import workloads as wl


def test_ppw_rule_reproduces_the_paper_grids():
    # Section 4.1: fourth-order operators, eps = 1e-4, domain size 2.25 give 318 x 318
    # unknowns at omega = 20 and 756 x 756 at omega = 40 (eq. NxFromPPW)
    assert int(wl.ppw_grid_points(20.0, order=4, eps=1e-4, size=2.25)) == 318
    assert int(wl.ppw_grid_points(40.0, order=4, eps=1e-4, size=2.25)) == 756


def test_ppw_rule_scaling():
    # N grows like omega^(1 + 1/p) and like eps^(-1/p)
    a = wl.ppw_grid_points(10.0, order=2, eps=1e-3)
    b = wl.ppw_grid_points(40.0, order=2, eps=1e-3)
    assert abs(b / a - 4.0 ** 1.5) < 1e-12
    c = wl.ppw_grid_points(10.0, order=2, eps=1e-5)
    assert abs(c / a - 10.0) < 1e-12
    # second order: b_1 = 2 (1!)^2 / 4! = 1/12
    assert abs(a - 10.0 * math.sqrt(10.0 / 12.0 / 2e-3)) < 1e-12


def test_ndsweep_problem_shape_and_source():
    q = wl.ndsweep_problem(12.0)
    assert q.n == math.ceil(wl.ppw_grid_points(12.0, 2, 1e-3))
    assert q.f.shape == (q.n + 1, q.n + 1)
    assert np.all(q.f[0] == 0) and np.all(q.f[:, -1] == 0)
    # peak omega^2 near x0 = (0.3, 0.4)
    j, i = np.unravel_index(np.argmax(q.f), q.f.shape)
    assert abs(i / q.n - 0.3) <= 1.0 / q.n and abs(j / q.n - 0.4) <= 1.0 / q.n
    assert q.f.max() <= 144.0 + 1e-9 and q.f.max() > 0.9 * 144.0


def test_compress_modes_round_trip():
    """The SVD compression of 2D nodal modes: exact rank for separable and rotated
    degenerate sine modes, reconstruction within the cut-off otherwise."""
    from compress_modes import compress_modes
    from oracle import modes
    n = 24
    a, b = modes.mode_nodal(2, n, (2, 5)), modes.mode_nodal(2, n, (5, 2))
    th = 0.3
    rot = np.cos(th) * a + np.sin(th) * b                     # same eigenvalue, rank 2
    rng = np.random.default_rng(3)
    g = rng.standard_normal((n + 1, n + 1))
    g[0] = g[-1] = 0
    g[:, 0] = g[:, -1] = 0
    V = np.stack([a, rot, g])
    fx, fy, tm, ranks = compress_modes(V, tol=1e-12)
    assert list(ranks[:2]) == [1, 2] and ranks[2] == n - 1
    assert list(tm) == [0] + [1] * 2 + [2] * int(ranks[2])
    for k in range(3):
        rec = sum(np.outer(fy[t], fx[t]) for t in range(len(tm)) if tm[t] == k)
        assert np.abs(rec - V[k]).max() < 1e-12 * np.abs(V[k]).max() * n
    # a loose cut-off keeps the leading singular values only; the error is bounded by them
    fx, fy, tm, ranks = compress_modes(V[2:], tol=0.3)
    s = np.linalg.svd(g, compute_uv=False)
    rec = sum(np.outer(fy[t], fx[t]) for t in range(len(tm)))
    assert ranks[0] == int(np.sum(s > 0.3 * s[0]))
    assert abs(np.linalg.norm(rec - g, 2) - s[ranks[0]]) < 1e-10 * s[0]
