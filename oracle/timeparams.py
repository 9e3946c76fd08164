"""Time-discretisation parameters of one wave solve (Section 2.2).

The explicit scheme (eq. discreteWaveExplicit) is stepped with time step dt over
Tbar = N_p periods, and the filter (eq. waveHoltzFilter) is approximated with
the trapezoid rule (eq. quadrature).  The paper removes the O(dt^2) time error
"by using an adjusted value for omega" in the wave solve and defers the formula
to earlier work; the reading taken here (R1) is:

    dt_cfl = cfl * h / c_max,   m = max(3, ceil(2 pi / (omega dt_cfl))),  N_t = N_p m,
    theta  = 2 pi / m,          dt = 2 sin(theta/2) / omega,
    omega_tilde = theta / dt    (used for the forcing, the filter and the period).

With these, U cos(omega_tilde t^n) solves the leapfrog recurrence exactly when
(L_h + omega^2) U = f, so the fixed point of Pi_h is the discrete Helmholtz
solution at the *given* omega.  ``freq_correction=False`` gives the uncorrected
reading (R2): dt = 2 pi/(m omega) and omega in the wave solve; its fixed point
solves L_h + omega_h^2 with omega_h = (2/dt) sin(omega dt/2).

Trapezoid weights: w_n = (2/Tbar) eta_n dt (cos(omega_tilde t^n) - 1/4),
eta_0 = eta_{N_t} = 1/2, else 1 (eq. quadrature, with cos(omega t) read as
cos(omega_tilde t^n) and the filter constant 1/4, i.e. alpha = 1/2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class TimeParams:
    omega: float          # Helmholtz frequency
    omega_w: float        # frequency used inside the wave solve (omega_tilde under R1)
    dt: float
    m: int                # steps per period
    nt: int               # N_t = N_p m
    n_periods: int
    tbar: float
    weights: np.ndarray   # w_n, n = 0..N_t
    forcing: np.ndarray   # cos(omega_w t^n), n = 0..N_t

    @property
    def omega_fixed_point(self) -> float:
        """The omega^2 whose discrete Helmholtz problem the fixed point solves."""
        return (2.0 / self.dt) * math.sin(self.omega_w * self.dt / 2.0)


def time_parameters(omega: float, h: float, c_max: float, cfl: float = 0.5,
                    n_periods: int = 1, steps_per_period: int = 0,
                    freq_correction: bool = True) -> TimeParams:
    if omega <= 0 or h <= 0 or c_max <= 0 or cfl <= 0 or n_periods < 1:
        raise ValueError("invalid time parameters")
    if steps_per_period:
        m = int(steps_per_period)
    else:
        dt_cfl = cfl * h / c_max
        m = max(3, int(math.ceil(2.0 * math.pi / (omega * dt_cfl))))
    if m < 3:
        raise ValueError("need at least 3 steps per period")
    nt = n_periods * m
    theta = 2.0 * math.pi / m
    if freq_correction:
        dt = 2.0 * math.sin(theta / 2.0) / omega
        omega_w = theta / dt
    else:
        dt = theta / omega
        omega_w = omega
    tbar = nt * dt
    n = np.arange(nt + 1)
    eta = np.ones(nt + 1)
    eta[0] = eta[-1] = 0.5
    forcing = np.cos(omega_w * n * dt)
    weights = (2.0 / tbar) * eta * dt * (forcing - 0.25)
    return TimeParams(omega, omega_w, dt, m, nt, n_periods, tbar, weights, forcing)
