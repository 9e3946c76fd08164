"""Pins of the oracle's deflation set and Krylov solvers: brute-force spectra,
the direct Helmholtz solve, algorithm invariants and the paper's stated rates."""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import discretization as disc, wavesolve as ws, transfer as tr, modes, krylov, devd
from _oracle_cases import setup, varc2

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _cfg(n=32, omega=21.3, dim=2, c2=None):
    L, tp, f = setup(dim, n, omega, c2=c2)
    U = disc.direct_solve(L, omega, f)
    b = ws.rhs(L, f, tp)
    A = lambda v: ws.apply_A(L, v, tp)
    return L, tp, f, U, b, A


def _err(x, U):
    return np.linalg.norm(x - U) / np.linalg.norm(U)


# ------------------------------------------------------------ modes
@pytest.mark.parametrize("dim,n", [(2, 12), (3, 6)])
def test_sine_modes_are_orthonormal_eigenvectors(dim, n):
    L = disc.laplacian(dim, n)
    ks = [(1, 1, 1), (2, 5, 1), (n - 1, 3, 2), (4, 4, 4)]
    ks = [k[:dim] for k in ks]
    W = modes.mode_matrix(dim, n, ks)
    lam2 = np.array([modes.mode_lam2(dim, n, k) for k in ks])
    assert np.abs(W.T @ W - np.eye(len(ks))).max() < 1e-14
    assert np.abs(L @ W + W * lam2).max() < 1e-10 * lam2.max()


def test_mode_selection_matches_brute_force():
    n, omega = 14, 27.0
    L = disc.laplacian(2, n)
    ev = np.sort(-np.linalg.eigvalsh(L.toarray()))
    sel, lam2 = modes.select_modes(2, n, omega, 6)
    # the selected lam2 are the 6 brute-force eigenvalues nearest omega^2
    brute = ev[np.argsort(np.abs(ev - omega ** 2), kind="stable")[:6]]
    assert np.allclose(np.sort(lam2), np.sort(brute), rtol=1e-12)
    # degenerate pairs (p,q)/(q,p) are both present and ordered lexicographically
    assert len(set(sel)) == 6
    for (p, q) in sel:
        if p != q and abs(modes.mode_lam2(2, n, (q, p)) - modes.mode_lam2(2, n, (p, q))) < 1e-9:
            assert (q, p) in sel


# ------------------------------------------------------------ FPI
def test_fpi_rate_is_max_abs_beta():
    # eq. WaveHoltzFPIconvergence: asymptotic rate = max_m |beta(lambda_m)|; with direct
    # deflation of the slowest modes it becomes the max over the remaining ones.
    n, omega = 16, 9.0
    L, tp, f = setup(2, n, omega)
    ev = np.linalg.eigvalsh(L.toarray())
    beta = tr.beta_discrete(-ev, tp)
    rho = np.max(np.abs(beta))
    b = ws.rhs(L, f, tp)
    _, info = krylov.fpi(lambda v: ws.wave_filter(L, v, f, tp), b, tol=1e-300, maxit=120)
    r = np.array(info["res"])
    obs = (r[-1] / r[-21]) ** (1 / 20)
    assert abs(obs - rho) < 5e-3
    # deflate the two slowest modes (DEVD with deflated forcing + iterates)
    sel, lam2 = modes.select_modes(2, n, omega, 5)
    W = modes.mode_matrix(2, n, sel)
    beta_m = tr.beta_discrete(lam2, tp)
    # remaining max after removing the deflated ones
    allb = list(np.abs(beta))
    for bm in np.abs(beta_m):
        allb.remove(min(allb, key=lambda x: abs(x - bm)))
    rho_d = max(allb)
    fd = devd.deflate(W, f)
    bd = ws.rhs(L, fd, tp)
    _, info = krylov.fpi(lambda v: devd.deflate(W, ws.wave_filter(L, v, fd, tp)), bd, tol=1e-300, maxit=50)
    r = np.array(info["res"])
    obs = (r[-1] / r[-21]) ** (1 / 20)     # still far above round-off at 50 iterations
    assert rho_d < rho and abs(obs - rho_d) < 5e-3


@pytest.mark.parametrize("deflate_iterates", [False, True])
def test_devd_fpi_matches_direct_solve_at_the_deflated_rate(deflate_iterates):
    # Algorithm 2 around the fixed-point iteration (devd_solve(method="fpi")): the inflated
    # result is the discrete Helmholtz solution, the iterates stay orthogonal to W, and the
    # observed rate is max |beta_h| over the modes that are not deflated
    # (eq. WaveHoltzFPIconvergence applied to the deflated problem).
    n, omega = 16, 9.0
    L, tp, f = setup(2, n, omega)
    U = disc.direct_solve(L, omega, f)
    ev = np.linalg.eigvalsh(L.toarray())
    beta = np.abs(tr.beta_discrete(-ev, tp))
    sel, lam2 = modes.select_modes(2, n, omega, 5)
    W = modes.mode_matrix(2, n, sel)
    rest = list(beta)
    for bm in np.abs(tr.beta_discrete(lam2, tp)):
        rest.remove(min(rest, key=lambda x: abs(x - bm)))
    rho_d = max(rest)
    assert rho_d < beta.max()
    x, info = devd.devd_solve(L, f, tp, W, lam2, method="fpi", tol=1e-12, maxit=2000,
                              deflate_iterates=deflate_iterates)
    assert _err(x, U) < 1e-10
    r = np.array(info["res"])
    k = len(r) - 1
    obs = (r[k] / r[k - 20]) ** (1 / 20)
    assert abs(obs - rho_d) < 5e-3, (obs, rho_d)
    # the deflated part of the solution is orthogonal to W; inflation restores W^T U
    v = devd.deflate(W, x)
    assert np.abs(W.T @ v).max() < 1e-13 * np.abs(x).max()
    assert np.abs(W.T @ x - W.T @ U).max() < 1e-10 * np.abs(W.T @ U).max()


def test_kappa_equals_condition_number_of_dense_A():
    # kappa_A = max|mu| / min|mu| over the spectrum {1 - beta_h(lambda)} equals the 2-norm
    # condition number of the dense A = I - S_h assembled column by column from wave solves
    for n, omega, c2 in [(10, 7.3, None), (9, 5.1, varc2(2, 9))]:
        L, tp, _ = setup(2, n, omega, c2=c2)
        A = ws.dense_A(L, tp)
        ev = np.linalg.eigvalsh(L.toarray())
        k_formula = tr.kappa(tr.mu_discrete(-ev, tp))
        k_dense = np.linalg.cond(A, 2)
        assert abs(k_formula - k_dense) < 1e-9 * k_dense, (k_formula, k_dense)
        # and kappa of the eigenvalues of the dense matrix itself
        assert abs(tr.kappa(np.linalg.eigvalsh(0.5 * (A + A.T))) - k_dense) < 1e-9 * k_dense


# ------------------------------------------------------------ CG / DCG
def test_beta_h_overshoot_window_is_small():
    # With the time-corrected frequency, beta_h peaks at 1 + O(dt^4) slightly below
    # omega, so A = I - S_h can be indefinite only for an eigenvalue inside a window
    # of relative width O(dt^2) below omega; above omega beta_h < 1.
    from oracle import timeparams as tpm
    for m in (20, 40, 80):
        tp = tpm.time_parameters(10.0, 1 / 512, 1.0, steps_per_period=m)
        z = np.linspace(-0.05, 0.05, 200001)
        b = tr.beta_discrete((10.0 * (1 + z)) ** 2, tp)
        over = z[b > 1 + 1e-15]
        assert b.max() - 1 < 4e-3 * (2 * math.pi / m) ** 4
        assert over.size == 0 or (over.max() <= 1e-12 and over.min() > -1.0 / m ** 2)
        assert np.all(b[z > 1e-9] < 1)


def test_cg_config1_matches_direct_solve():
    p = wl.config1()
    L, tp, f = setup(2, p.n, p.omega, f=p.f)
    U = disc.direct_solve(L, p.omega, f)
    b = ws.rhs(L, f, tp)
    x, info = krylov.cg(lambda v: ws.apply_A(L, v, tp), b, tol=1e-10)
    assert _err(x, U) < 1e-10
    assert info["res"][-1] <= 1e-10
    true = np.linalg.norm(b - ws.apply_A(L, x, tp)) / np.linalg.norm(b)
    assert abs(true - info["res"][-1]) < 1e-11


def test_cg_variable_c_3d():
    c2 = varc2(3, 10, seed=5)
    L, tp, f, U, b, A = _cfg(10, 8.3, 3, c2)
    x, _ = krylov.cg(A, b, tol=1e-12)
    assert _err(x, U) < 1e-10


def _near_resonant():
    # omega placed just below a discrete eigenvalue so that deflation matters (and
    # outside the narrow window just *below* omega where beta_h exceeds 1)
    n = 32
    lam = math.sqrt(modes.mode_lam2(2, n, (5, 6)))
    return _cfg(n, lam * (1 - 2e-3))


def test_dcg_invariants_and_solution():
    L, tp, f, U, b, A = _near_resonant()
    sel, lam2 = modes.select_modes(2, 32, tp.omega, 8)
    W = modes.mode_matrix(2, 32, sel)
    mu = tr.mu_discrete(lam2, tp)
    x, info = krylov.dcg(A, b, W, W * mu, tol=1e-11)
    xc, infc = krylov.cg(A, b, tol=1e-11)
    assert _err(x, U) < 1e-9 and _err(xc, U) < 1e-9
    # W^T r_k = 0 for every k (Section 3.1: the deflated start and the projections)
    assert max(info["wtr"]) < 1e-12 * np.linalg.norm(b)
    assert info["iters"] < infc["iters"]
    # without re-projection it still converges with exact eigenvectors (Section 3.1)
    x2, info2 = krylov.dcg(A, b, W, W * mu, tol=1e-11, reproject=False)
    assert _err(x2, U) < 1e-9 and abs(info2["iters"] - info["iters"]) <= 2


def test_dcg_with_general_vectors():
    # Algorithm 3 with vectors that are not eigenvectors (perturbed sine modes, re-orthonormalised):
    # A W costs wave solves, (W^T A W) is dense, and the per-iteration A-orthogonalisation is
    # what keeps W^T r_k = 0; the iterate still converges to the discrete Helmholtz solution
    L, tp, f, U, b, A = _near_resonant()
    sel, lam2 = modes.select_modes(2, 32, tp.omega, 8)
    E = modes.mode_matrix(2, 32, sel)
    rng = np.random.default_rng(3)
    W, _ = np.linalg.qr(E + 1e-3 * rng.standard_normal(E.shape) / np.sqrt(E.shape[0]))
    AW = np.column_stack([A(W[:, k]) for k in range(W.shape[1])])
    assert np.abs(W.T @ AW - (W.T @ AW).T).max() < 1e-12     # W^T A W symmetric (A symmetric)
    x, info = krylov.dcg(A, b, W, AW, tol=1e-11)
    assert _err(x, U) < 1e-9
    assert max(info["wtr"]) < 1e-10 * np.linalg.norm(b)
    _, infc = krylov.cg(A, b, tol=1e-11)
    _, infe = krylov.dcg(A, b, E, E * tr.mu_discrete(lam2, tp), tol=1e-11)
    assert infe["iters"] <= info["iters"] < infc["iters"]
    # dropping the re-projection (allowed only for eigenvectors) loses the invariant
    _, info2 = krylov.dcg(A, b, W, AW, tol=1e-11, maxit=40, reproject=False)
    assert max(info2["wtr"]) > 1e3 * max(info["wtr"])


def test_dcg_error_bound_theorem():
    # Theorem 3.1 with kappa_D of Theorem 3.2 on a dense A
    n, omega = 10, 13.0
    L, tp, f = setup(2, n, omega)
    Ad = ws.dense_A(L, tp)
    Ad = 0.5 * (Ad + Ad.T)
    evals, evecs = np.linalg.eigh(Ad)
    nd = 5
    W = evecs[:, :nd]
    kd = evals[-1] / evals[nd]
    assert abs(tr.kappa_deflated(evals, nd) - kd) < 1e-12
    rate = tr.dcg_rate(kd)
    b = Ad @ np.random.default_rng(0).standard_normal(Ad.shape[0])
    xs = np.linalg.solve(Ad, b)
    errA = lambda x: math.sqrt((x - xs) @ Ad @ (x - xs))
    for j in range(1, 12):
        x, _ = krylov.dcg(lambda v: Ad @ v, b, W, Ad @ W, tol=0, maxit=j)
        x0, _ = krylov.dcg(lambda v: Ad @ v, b, W, Ad @ W, tol=0, maxit=0)
        assert errA(x) <= 2 * rate ** j * errA(x0) * (1 + 1e-8) + 1e-13


def test_paper_kappa3_rate():
    g = GOLD["dcg_kappa3"]
    k = g["mu_max"] / g["mu_deflated_max"]
    assert k == g["kappa_D"]
    rate = tr.dcg_rate(k)
    assert round(rate, g["rate_digits"]) == g["rate"]
    for its, orders in g["orders"]:
        assert 2 * rate ** its <= 10.0 ** (-orders)


# ------------------------------------------------------------ GMRES / AGMRES / BiCGStab
def test_gmres_givens_residual_is_true_residual():
    n, omega = 10, 13.0
    L, tp, f = setup(2, n, omega)
    Ad = ws.dense_A(L, tp)
    b = ws.rhs(L, f, tp)
    nb = np.linalg.norm(b)
    for k in (1, 3, 7, 15):
        x, info = krylov.agmres(lambda v: Ad @ v, b, restart=40, tol=0, maxit=k)
        assert abs(info["gres"][-1] - np.linalg.norm(b - Ad @ x) / nb) < 1e-12


@pytest.mark.parametrize("restart", [5, 40])
def test_gmres_restarted_matches_direct_solve(restart):
    L, tp, f, U, b, A = _cfg(24, 17.1)
    x, info = krylov.agmres(A, b, restart=restart, tol=1e-11, maxit=2000)
    assert _err(x, U) < 1e-9


def test_agmres_augmented_with_eigenvectors():
    L, tp, f, U, b, A = _near_resonant()
    sel, lam2 = modes.select_modes(2, 32, tp.omega, 8)
    W = modes.mode_matrix(2, 32, sel)
    AW = W * tr.mu_discrete(lam2, tp)
    x, info = krylov.agmres(A, b, W=W, AW=AW, restart=40, tol=1e-11, maxit=500)
    xg, infg = krylov.agmres(A, b, restart=40, tol=1e-11, maxit=500)
    assert _err(x, U) < 1e-9
    # restarted GMRES(40) stagnates near resonance; augmentation removes the slow modes
    assert info["iters"] < infg["iters"] and _err(x, U) < _err(xg, U)


def test_abicgstab_augmented():
    L, tp, f, U, b, A = _near_resonant()
    sel, lam2 = modes.select_modes(2, 32, tp.omega, 8)
    W = modes.mode_matrix(2, 32, sel)
    AW = W * tr.mu_discrete(lam2, tp)
    x, info = krylov.abicgstab(A, b, W=W, AW=AW, tol=1e-11, maxit=500)
    assert _err(x, U) < 1e-8


# ------------------------------------------------------------ DEVD
def test_devd_matches_direct_solve_and_inflation_is_exact():
    L, tp, f, U, b, A = _near_resonant()
    sel, lam2 = modes.select_modes(2, 32, tp.omega, 8)
    W = modes.mode_matrix(2, 32, sel)
    x, info = devd.devd_solve(L, f, tp, W, lam2, tol=1e-11)
    assert _err(x, U) < 1e-9
    # a forcing inside span(W): the deflated problem is zero and inflation alone is exact
    f2 = W @ np.arange(1.0, 9.0)
    U2 = disc.direct_solve(L, tp.omega, f2)
    x2 = devd.inflate(W, lam2, tp.omega, f2, np.zeros_like(f2))
    assert _err(x2, U2) < 1e-12


def test_resonant_omega_makes_A_singular_and_krylov_stalls():
    """At omega^2 equal to the discrete eigenvalue lambda_{1,1} of -L_h the filter passes that mode
    unchanged (mu = 1 - beta_h = 0 up to rounding, the exactness the omega-tilde correction of
    eq. R1 gives), so A = I - S_h is singular with b outside its range: neither CG nor GMRES may
    report convergence.  The GPU solvers' failure status is tested against the same system."""
    n = 16
    lam2 = modes.mode_lam2(2, n, (1, 1))
    om = math.sqrt(lam2)
    L, tp, f = setup(2, n, om)
    assert abs(tr.mu_discrete(np.array([lam2]), tp)[0]) < 1e-12
    # the (1,1) mode is a null vector of A
    v = disc.to_interior(modes.mode_nodal(2, n, (1, 1)))
    Av = ws.apply_A(L, v, tp)
    assert np.linalg.norm(Av) < 1e-12 * np.linalg.norm(v)
    b = ws.rhs(L, f, tp)
    A = lambda x: ws.apply_A(L, x, tp)
    _, ci = krylov.cg(A, b, tol=1e-10, maxit=300)
    _, gi = krylov.agmres(A, b, tol=1e-10, maxit=300)
    assert ci["iters"] == 300 and ci["res"][-1] > 1e-10
    assert gi["iters"] >= 300 and gi["res"][-1] > 1e-10
