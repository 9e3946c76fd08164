"""The discrete WaveHoltz filter operator Pi_h (Section 2.2).

One "wave solve" (eq. WaveHoltzDiscreteFPI): step the explicit scheme
(eq. discreteWaveExplicit)

    W^0 = v,   D_{0t} W^0 = 0,
    W^{n+1} = 2 W^n - W^{n-1} + dt^2 (L_h W^n - f cos(omega_w t^n)),  n = 0..N_t-1,

where D_{0t} W^0 = 0 means W^{-1} = W^1, so the first step is
W^1 = W^0 + dt^2/2 (L_h W^0 - f), and accumulate the trapezoid filter
(eq. quadrature)  Pi_h v = sum_{n=0}^{N_t} w_n W^n.

Then b = Pi_h 0 and A v = (I - S_h) v = v - Pi_h(v; f=0)  (eq. I_minus_S).
"""
from __future__ import annotations

import numpy as np

from .timeparams import TimeParams


def wave_filter(L, v: np.ndarray, f: np.ndarray | None, tp: TimeParams,
                state_dtype=np.float64, trajectory: list | None = None) -> np.ndarray:
    """Pi_h(v; f).  ``state_dtype=np.float32`` stores W^n in single precision while the
    filter sum stays in double (used only to predict the size of mixed-precision error).
    If ``trajectory`` is a list, every W^n (n = 0..N_t) is appended to it."""
    dt2 = tp.dt * tp.dt
    sd = state_dtype
    Lc = L.astype(sd) if sd != np.float64 else L
    fz = None if f is None else np.asarray(f, dtype=sd)
    W0 = np.asarray(v, dtype=sd).copy()
    LW = Lc @ W0
    if fz is not None:
        LW = LW - fz * sd(tp.forcing[0])
    W1 = (W0 + sd(0.5 * dt2) * LW).astype(sd)
    V = tp.weights[0] * W0.astype(np.float64) + tp.weights[1] * W1.astype(np.float64)
    if trajectory is not None:
        trajectory.append(W0.astype(np.float64)); trajectory.append(W1.astype(np.float64))
    for n in range(1, tp.nt):
        LW = Lc @ W1
        if fz is not None:
            LW = LW - fz * sd(tp.forcing[n])
        W2 = (sd(2) * W1 - W0 + sd(dt2) * LW).astype(sd)
        V += tp.weights[n + 1] * W2.astype(np.float64)
        if trajectory is not None:
            trajectory.append(W2.astype(np.float64))
        W0, W1 = W1, W2
    return V


def rhs(L, f, tp: TimeParams, **kw) -> np.ndarray:
    """b = Pi_h 0."""
    return wave_filter(L, np.zeros(L.shape[0]), f, tp, **kw)


def apply_S(L, v, tp: TimeParams, **kw) -> np.ndarray:
    """S_h v = Pi_h(v) - Pi_h(0) = Pi_h(v; f = 0)."""
    return wave_filter(L, v, None, tp, **kw)


def apply_A(L, v, tp: TimeParams, **kw) -> np.ndarray:
    """A v = (I - S_h) v."""
    return np.asarray(v, dtype=np.float64) - apply_S(L, v, tp, **kw)


def dense_A(L, tp: TimeParams) -> np.ndarray:
    """A built column by column by applying it to unit vectors (tiny grids only)."""
    N = L.shape[0]
    A = np.empty((N, N))
    e = np.zeros(N)
    for j in range(N):
        e[j] = 1.0
        A[:, j] = apply_A(L, e, tp)
        e[j] = 0.0
    return A


def apply_A_defect(L, v, tp: TimeParams, **kw) -> np.ndarray:
    """A v computed as B (L_h + omega^2) v with B f = Pi_h(0; f).

    With the corrected frequency, a trajectory started at W^0 = v splits as
    W^n = cos(omega_w t^n) v + E^n, where E solves the same scheme from zero data with
    forcing (L_h + omega^2) v in place of -f (the term cos(n theta) v absorbs the rest
    because (2/dt^2)(cos theta - 1) = -omega^2), and the trapezoid weights integrate
    cos^2 to one, so  A v = v - Pi_h(v; 0) = -sum_n w_n E^n = Pi_h(0; (L_h + omega^2) v).
    Stepping E instead of W keeps rounding errors proportional to |E|, which is small
    for the near-resonant components of v."""
    g = L @ v + tp.omega ** 2 * np.asarray(v, dtype=np.float64)
    return wave_filter(L, np.zeros(L.shape[0]), -g, tp, **kw) * -1.0
