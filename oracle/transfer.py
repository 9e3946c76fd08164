"""Filter transfer functions (Section 2.3).

Continuous (eq. beta_fun):
    beta(lam; omega) = (2/Tbar) int_0^Tbar (cos(omega t) - 1/4) cos(lam t) dt
                     = sinc(omega+lam) + sinc(omega-lam) - 1/2 sinc(lam),
with sinc(x) read as sin(x Tbar)/(x Tbar) (value 1 at x = 0) and Tbar = N_p 2 pi/omega.

Discrete (exact for the scheme of Section 2.2): for an eigenvector of L_h with
L_h Phi = -lam2 Phi, the leapfrog recurrence with the half first step gives
W^n = T_n(1 - lam2 dt^2/2) Phi (T_n the Chebyshev polynomial, = cos(n theta_lam)
when stable), hence S_h Phi = beta_h(lam2) Phi with
    beta_h(lam2) = sum_n w_n T_n(1 - lam2 dt^2 / 2).
The eigenvalues of A = I - S_h are mu = 1 - beta (eq. eigenvaluesOfM).
"""
from __future__ import annotations

import math

import numpy as np

from .timeparams import TimeParams


def sinc_T(x, tbar):
    x = np.asarray(x, dtype=np.float64) * tbar
    out = np.ones_like(x)
    nz = np.abs(x) > 0
    out[nz] = np.sin(x[nz]) / x[nz]
    return out


def beta_continuous(lam, omega: float, n_periods: int = 1):
    tbar = n_periods * 2.0 * math.pi / omega
    lam = np.asarray(lam, dtype=np.float64)
    return sinc_T(omega + lam, tbar) + sinc_T(omega - lam, tbar) - 0.5 * sinc_T(lam, tbar)


def chebyshev_T(n_max: int, x):
    """T_0..T_{n_max} at x by the three-term recurrence; shape (n_max+1, *x.shape)."""
    x = np.asarray(x, dtype=np.float64)
    T = np.empty((n_max + 1,) + x.shape)
    T[0] = 1.0
    if n_max >= 1:
        T[1] = x
    for k in range(1, n_max):
        T[k + 1] = 2.0 * x * T[k] - T[k - 1]
    return T


def beta_discrete(lam2, tp: TimeParams):
    """beta_h for discrete eigenvalues lam2 = lambda_h^2 of -L_h."""
    lam2 = np.asarray(lam2, dtype=np.float64)
    T = chebyshev_T(tp.nt, 1.0 - 0.5 * lam2 * tp.dt ** 2)
    return np.tensordot(tp.weights, T, axes=(0, 0))


def mu_discrete(lam2, tp: TimeParams):
    """Eigenvalues of A = I - S_h on the eigenvectors with eigenvalue lam2."""
    return 1.0 - beta_discrete(lam2, tp)


def c_beta(n_periods: int) -> float:
    """C_beta in beta = 1 - C_beta z^2 + O(z^3), z = (lam-omega)/omega (eq. betaGap)."""
    return (2.0 / 3.0) * n_periods ** 2 * math.pi ** 2 - 0.25


def kappa(mu) -> float:
    """kappa_A = max|mu| / min|mu| (Section 2.3)."""
    a = np.abs(np.asarray(mu))
    return float(a.max() / a.min())


def kappa_deflated(mu_sorted_all, n_defl: int) -> float:
    """kappa_D = mu_N / mu_{N_D+1} for the mu's sorted ascending, deflating the
    N_D smallest (Theorem 3.2)."""
    m = np.sort(np.asarray(mu_sorted_all))
    return float(m[-1] / m[n_defl])


def dcg_rate(kappa_d: float) -> float:
    """(sqrt(kappa)-1)/(sqrt(kappa)+1), the per-iteration factor of Theorem 3.1."""
    s = math.sqrt(kappa_d)
    return (s - 1.0) / (s + 1.0)
