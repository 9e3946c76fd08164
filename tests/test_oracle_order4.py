"""Pins of the oracle's fourth-order operator (c = 1, odd reflection at the Dirichlet
boundary) against closed forms and the mathematics of the scheme."""
import numpy as np
import pytest

from oracle import discretization as disc, modes, timeparams as tpm, wavesolve as ws

pytestmark = pytest.mark.filterwarnings("ignore")


@pytest.mark.parametrize("dim,n", [(2, 12), (3, 7)])
def test_sine_vectors_are_eigenvectors(dim, n):
    # the boundary rows included: every sine vector, with the closed-form eigenvalue
    L = disc.laplacian(dim, n, order=4)
    for idx in [(1,) * dim, (n - 1, 2, 3)[:dim], (2, n - 2, 1)[:dim]]:
        phi = disc.to_interior(modes.mode_nodal(dim, n, idx))
        lam2 = modes.mode_lam2(dim, n, idx, order=4)
        t = np.array(idx) * np.pi / n
        closed = float(np.sum((30 - 32 * np.cos(t) + 2 * np.cos(2 * t)) * n * n / 12.0))
        assert abs(lam2 - closed) < 1e-12 * closed
        assert np.abs(L @ phi + lam2 * phi).max() < 1e-9 * lam2


def test_symmetric_and_fourth_order_consistent():
    L = disc.laplacian(2, 16, order=4)
    assert abs(L - L.T).max() < 1e-12
    # u = sin(pi x) sin(2 pi y): odd about every boundary, so the reflection closure is
    # exact to the interior order; the truncation error falls by 2^4 per halving of h
    errs = []
    for n in (16, 32, 64):
        x = np.arange(n + 1) / n
        X, Y = np.meshgrid(x, x, indexing="xy")
        u = np.sin(np.pi * X) * np.sin(2 * np.pi * Y)
        Lu = disc.laplacian(2, n, order=4) @ disc.to_interior(u)
        errs.append(np.abs(Lu + 5 * np.pi ** 2 * disc.to_interior(u)).max())
    assert 14 < errs[0] / errs[1] < 18 and 14 < errs[1] / errs[2] < 18
    # the second-order operator only reaches 2^2
    n = 32
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = np.sin(np.pi * X) * np.sin(2 * np.pi * Y)
    e2 = np.abs(disc.laplacian(2, n) @ disc.to_interior(u) + 5 * np.pi ** 2 * disc.to_interior(u)).max()
    assert e2 > 50 * errs[1]


def test_dst_solve_matches_sparse_lu():
    n, omega = 40, 13.7
    rng = np.random.default_rng(4)
    f = np.zeros((n + 1, n + 1))
    f[1:-1, 1:-1] = rng.standard_normal((n - 1, n - 1))
    U = disc.direct_solve_dst(2, n, omega, f, order=4)
    U2 = disc.direct_solve(disc.laplacian(2, n, order=4), omega, disc.to_interior(f))
    assert np.abs(disc.to_interior(U) - U2).max() < 1e-11 * np.abs(U2).max()


def test_time_corrected_fixed_point_with_fourth_order():
    # Pi_h U* = U* holds for any symmetric L_h under the adjusted frequency
    n, omega = 24, 9.1
    L = disc.laplacian(2, n, order=4)
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    f = np.exp(-((X - 0.4) ** 2 + (Y - 0.55) ** 2) / 0.02)
    f[0] = f[-1] = 0
    f[:, 0] = f[:, -1] = 0
    U = disc.direct_solve(L, omega, disc.to_interior(f))
    tp = tpm.time_parameters(omega, 1.0 / n, 1.0, cfl=0.5)
    V = ws.wave_filter(L, U, disc.to_interior(f), tp)
    assert np.abs(V - U).max() < 1e-12 * np.abs(U).max()


def test_mode_selection_by_order():
    # the two spectra part at high k (the fourth-order one lies above): the selected sets
    # differ for a high frequency, and each is sorted by its own distance
    n, omega = 32, 60.0
    s2, l2 = modes.select_modes(2, n, omega, 12)
    s4, l4 = modes.select_modes(2, n, omega, 12, order=4)
    assert s2 != s4
    d4 = np.abs(np.asarray(l4) - omega ** 2)
    assert np.all(np.diff(d4) >= -1e-9 * omega ** 2)
    assert all(abs(modes.mode_lam2(2, n, m, order=4) - l) < 1e-9 for m, l in zip(s4, l4))
