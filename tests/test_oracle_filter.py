"""Pins of the oracle's time parameters, filter operator and transfer functions
against closed forms, the direct Helmholtz solve and the paper's stated values."""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

import workloads as wl
from oracle import discretization as disc, timeparams as tpm, wavesolve as ws, transfer as tr, modes
from _oracle_cases import setup, varc2

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# ------------------------------------------------------------ time parameters
@pytest.mark.parametrize("omega,n,cfl", [(20.5, 64, 0.5), (100.3, 1024, 0.5), (40.0, 256, 0.5), (7.3, 16, 0.3)])
def test_time_params_r1_identities(omega, n, cfl):
    tp = tpm.time_parameters(omega, 1.0 / n, 1.0, cfl=cfl)
    dt_cfl = cfl / n
    assert tp.m == max(3, math.ceil(2 * math.pi / (omega * dt_cfl)))
    assert tp.dt <= dt_cfl * (1 + 1e-15)
    # omega_tilde dt = 2 pi / m and the leapfrog dispersion maps omega_tilde to omega
    assert abs(tp.omega_w * tp.dt - 2 * math.pi / tp.m) < 1e-14
    assert abs((2 / tp.dt) * math.sin(tp.omega_w * tp.dt / 2) - omega) < 1e-12 * omega
    assert abs(tp.tbar - 2 * math.pi / tp.omega_w) < 1e-13


def test_weights_integrate_whole_periods():
    # trapezoid over whole periods: sum_n eta_n cos(n theta) = 0 and sum eta cos^2 = N_t/2 (m >= 3)
    for m in (3, 4, 7, 40):
        tp = tpm.time_parameters(10.0, 1 / 64, 1.0, steps_per_period=m, n_periods=2)
        assert abs(tp.weights.sum() + 0.5) < 1e-13           # (2/T) int (cos - 1/4) = -1/2
        assert abs(tp.weights @ tp.forcing - 1.0) < 1e-13    # (2/T) int (cos - 1/4) cos = 1


def test_config1_time_parameters():
    tp = tpm.time_parameters(20.5, 1 / 64, 1.0, cfl=0.5)
    assert tp.m == 40 and tp.nt == 40


# ------------------------------------------------------------ fixed point
@pytest.mark.parametrize("case", ["cfg1", "2d-varc", "3d-varc", "2d-np2"])
def test_fixed_point_is_direct_solution(case):
    if case == "cfg1":
        p = wl.config1()
        L, tp, f = setup(2, p.n, p.omega, f=p.f)
    elif case == "2d-varc":
        c2 = varc2(2, 40)
        L, tp, f = setup(2, 40, 17.3, c2=c2)
    elif case == "3d-varc":
        c2 = varc2(3, 12, seed=3)
        L, tp, f = setup(3, 12, 9.1, c2=c2)
    else:
        L, tp, f = setup(2, 32, 13.7, n_periods=2)
    U = disc.direct_solve(L, tp.omega, f)
    PU = ws.wave_filter(L, U, f, tp)
    assert np.linalg.norm(PU - U) / np.linalg.norm(U) < 1e-13


def test_uncorrected_reading_fixed_point():
    # R2: wave solve at omega itself; the fixed point solves L_h + omega_h^2
    L, tp, f = setup(2, 48, 21.0, freq_correction=False)
    assert tp.omega_w == 21.0
    U = disc.direct_solve(L, tp.omega_fixed_point, f)
    assert np.linalg.norm(ws.wave_filter(L, U, f, tp) - U) / np.linalg.norm(U) < 1e-13
    # ... and it differs from the corrected answer by O(dt^2) (not a cosmetic change)
    U1 = disc.direct_solve(L, 21.0, f)
    assert np.linalg.norm(U - U1) / np.linalg.norm(U1) > 1e-4


def test_trajectory_at_fixed_point_is_time_harmonic():
    L, tp, f = setup(2, 24, 11.2)
    U = disc.direct_solve(L, tp.omega, f)
    traj = []
    ws.wave_filter(L, U, f, tp, trajectory=traj)
    for k, Wk in enumerate(traj):
        assert np.linalg.norm(Wk - U * math.cos(tp.omega_w * k * tp.dt)) < 1e-12 * np.linalg.norm(U)


# ------------------------------------------------------------ transfer functions
@pytest.mark.parametrize("dim,n,omega", [(2, 32, 15.2), (3, 10, 8.7)])
def test_filter_acts_on_modes_by_beta_h(dim, n, omega):
    L, tp, _ = setup(dim, n, omega)
    idxs = [(1, 1, 1)[:dim], (3, 2, 1)[:dim], (n - 1, 2, 3)[:dim], (n - 1, n - 1, n - 1)[:dim]]
    for idx in idxs:
        phi = disc.to_interior(modes.mode_nodal(dim, n, idx))
        lam2 = modes.mode_lam2(dim, n, idx)
        Sphi = ws.apply_S(L, phi, tp)
        assert np.linalg.norm(Sphi - tr.beta_discrete(lam2, tp) * phi) < 1e-13


def test_beta_h_is_one_at_resonance():
    tp = tpm.time_parameters(33.3, 1 / 128, 1.0)
    assert abs(tr.beta_discrete(33.3 ** 2, tp) - GOLD["beta_at_omega"]["value"]) < 1e-13
    assert abs(tr.beta_continuous(33.3, 33.3) - 1.0) < 1e-14


def test_sinc_reading_matches_defining_integral():
    # beta(lam; omega) = (2/T) int_0^T (cos(omega t) - 1/4) cos(lam t) dt
    for Np in (1, 2, 3):
        om = 5.0
        T = Np * 2 * math.pi / om
        for lam in (0.0, 1.3, 4.9, 5.0, 7.7, 15.1):
            val = quad(lambda t: (math.cos(om * t) - 0.25) * math.cos(lam * t), 0, T, limit=200)[0] * 2 / T
            assert abs(tr.beta_continuous(lam, om, Np) - val) < 1e-10


def test_beta_h_converges_to_beta_as_dt_shrinks():
    # beta_h(lam^2) -> beta(lam; omega) at second order in dt
    om, lam = 10.0, 9.3
    errs = []
    for m in (20, 40, 80, 160):
        tp = tpm.time_parameters(om, 1 / 512, 1.0, steps_per_period=m)
        errs.append(abs(tr.beta_discrete(lam ** 2, tp) - tr.beta_continuous(lam, om)))
    for a, b in zip(errs, errs[1:]):
        assert 3.0 < a / b < 5.0


@pytest.mark.parametrize("Np", [1, 2, 3])
def test_c_beta_expansion(Np):
    g = GOLD["c_beta"]
    cb = g["coef_np2_pi2"] * Np ** 2 * math.pi ** 2 + g["offset"]
    assert abs(tr.c_beta(Np) - cb) < 1e-12
    om = 7.0
    for z in (1e-3, -1e-3):
        est = (1 - tr.beta_continuous(om * (1 + z), om, Np)) / z ** 2
        assert abs(est - cb) / cb < 5e-3


def test_beta_lower_bound_and_mu_upper_bound():
    g = GOLD["beta_lower_bound"]
    lam = np.linspace(0, 50, 200001)
    for Np in (1, 2, 3):
        b = tr.beta_continuous(lam, 5.0, Np)
        assert b.min() >= g["beta_min"] - 1e-12
        assert (1 - b).max() <= g["mu_max"] + 1e-12
    assert abs(tr.beta_continuous(0.0, 5.0) - (-0.5)) < 1e-15


@pytest.mark.parametrize("omega,n,cfl", [(5.3, 64, 0.5), (17.1, 64, 0.5), (40.0, 128, 0.5), (23.4, 96, 0.7)])
def test_discrete_beta_bounded_for_a_stable_step(omega, n, cfl):
    """With a stable leapfrog step (c dt/h below 1/sqrt(2) in 2D) the discrete filter's
    eigenvalue beta_h stays in [-1/2, 1 + O(dt^4)] over the whole 2D spectrum
    lambda^2 in [0, 8/h^2], so |A| <= 1.5 (the bound the solvers test for instability);
    beyond the CFL bound it leaves that range by orders of magnitude."""
    h = 1.0 / n
    tp = tpm.time_parameters(omega, h, 1.0, cfl=cfl)
    lam2 = np.linspace(0.0, 8.0 / h ** 2, 400001)
    b = tr.beta_discrete(lam2, tp)
    assert b.min() >= -0.5 - 1e-12 and b.max() <= 1.0 + 1e-3
    assert np.abs(1.0 - b).max() <= 1.5 + 1e-12
    # the same time step applied to c = 2 (an understated c_max of 1): unstable
    bu = tr.beta_discrete(4.0 * lam2, tp)
    assert np.abs(bu).max() > 1e6


# ------------------------------------------------------------ the matrix A
@pytest.mark.parametrize("dim,n,omega,varc", [(2, 8, 6.1, False), (2, 8, 6.1, True), (3, 5, 5.3, True)])
def test_dense_A_symmetric_spectrum(dim, n, omega, varc):
    c2 = varc2(dim, n) if varc else None
    L, tp, _ = setup(dim, n, omega, c2=c2)
    A = ws.dense_A(L, tp)
    assert np.abs(A - A.T).max() < 1e-13
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    lam2 = -np.linalg.eigvalsh(L.toarray())
    mu = np.sort(tr.mu_discrete(lam2, tp))
    assert np.abs(np.sort(ev) - mu).max() < 1e-12
    assert ev.min() > 0   # SPD off resonance
    if not varc:
        # the analytic spectrum of the constant-coefficient Laplacian
        e1 = modes.eig1d(n)
        an = np.sort(np.add.outer(e1, e1).ravel() if dim == 2 else
                     np.add.outer(np.add.outer(e1, e1), e1).ravel())
        assert np.abs(np.sort(lam2) - an).max() < 1e-10 * an.max()


def test_mixed_precision_error_size():
    # FP32 stepping with an FP64 filter sum: operator error ~1e-6 relative (predicts the mixed path)
    L, tp, f = setup(2, 64, 20.5)
    v = disc.to_interior(wl.random_nodal(2, 64, 1))
    e = np.linalg.norm(ws.apply_S(L, v, tp, state_dtype=np.float32) - ws.apply_S(L, v, tp)) / np.linalg.norm(v)
    assert 1e-9 < e < 1e-5


@pytest.mark.parametrize("dim,n,omega", [(2, 40, 17.3), (3, 9, 6.2)])
def test_dst_direct_solve_matches_sparse_lu(dim, n, omega):
    f = wl.gaussian(dim, n, (0.3, 0.6, 0.5)[:dim], 0.1)
    L = disc.laplacian(dim, n)
    U = disc.to_nodal(disc.direct_solve(L, omega, disc.to_interior(f)), dim, n)
    assert np.abs(disc.direct_solve_dst(dim, n, omega, f) - U).max() < 1e-12 * np.abs(U).max()


@pytest.mark.parametrize("dim,n,omega,varc", [(2, 32, 13.7, False), (2, 24, 9.3, True), (3, 8, 6.1, True)])
def test_A_equals_B_times_helmholtz_operator(dim, n, omega, varc):
    # A = I - S_h = B H with B f = Pi_h(0; f) and H = L_h + omega^2 (corrected frequency)
    c2 = varc2(dim, n) if varc else None
    L, tp, _ = setup(dim, n, omega, c2=c2)
    v = disc.to_interior(wl.random_nodal(dim, n, 3))
    a1 = ws.apply_A(L, v, tp)
    a2 = ws.apply_A_defect(L, v, tp)
    assert np.linalg.norm(a1 - a2) < 1e-12 * np.linalg.norm(a1)
    # with the uncorrected frequency the identity fails (it relies on the dispersion match)
    tp2 = tpm.time_parameters(omega, 1.0 / n, 1.0 if c2 is None else float(np.sqrt(c2.max())),
                              freq_correction=False)
    assert np.linalg.norm(ws.apply_A(L, v, tp2) - ws.apply_A_defect(L, v, tp2)) > 1e-6 * np.linalg.norm(a1)


@pytest.mark.parametrize("mode", [(5, 6), (3, 7), (8, 2)])
@pytest.mark.parametrize("gap", [1e-3, 1e-2])
def test_defect_form_reduces_fp32_error_near_resonance(mode, gap):
    # FP32 stepping of W versus FP32 stepping of the defect E on a near-resonant eigenvector,
    # where A's eigenvalue mu = 1 - beta_h is small (Section 2.3): in the W form the rounding
    # of W ~ |v| is divided by mu when A v = v - Pi v is formed, in the defect form the stepped
    # state is E ~ mu |v| itself, so the relative error of A v drops by a large factor
    n = 64
    lam2 = modes.mode_lam2(2, n, mode)
    omega = np.sqrt(lam2) * (1 - gap)
    L, tp, _ = setup(2, n, omega)
    phi = disc.to_interior(modes.mode_nodal(2, n, mode))
    a = ws.apply_A(L, phi, tp)
    e_w = np.linalg.norm(ws.apply_A(L, phi, tp, state_dtype=np.float32) - a) / np.linalg.norm(a)
    e_e = np.linalg.norm(ws.apply_A_defect(L, phi, tp, state_dtype=np.float32) - a) / np.linalg.norm(a)
    assert e_e < e_w / 20, (e_e, e_w)
    assert e_e < 3e-5


@pytest.mark.parametrize("dim,n,omega,varc", [(2, 20, 11.3, False), (2, 16, 7.7, True), (3, 7, 5.2, True)])
def test_helmholtz_residual_of_a_perturbed_solve(dim, n, omega, varc):
    # U solving (L_h + omega^2) U = f + d has residual exactly ||d|| / ||f|| against f
    c2 = varc2(dim, n) if varc else None
    L = disc.laplacian(dim, n, c2)
    f = disc.to_interior(wl.gaussian(dim, n, (0.4, 0.6, 0.5)[:dim], 0.15))
    d = 1e-3 * disc.to_interior(wl.random_nodal(dim, n, 5))
    U = disc.direct_solve(L, omega, f + d)
    want = np.linalg.norm(d) / np.linalg.norm(f)
    assert abs(disc.helmholtz_residual(L, omega, U, f) - want) < 1e-8 * want
    assert disc.helmholtz_residual(L, omega, disc.direct_solve(L, omega, f), f) < 1e-12
