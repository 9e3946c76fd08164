"""Gradient of a receiver misfit with respect to the nodal c^2.

Misfit J(c2) = 1/2 sum_s ||R u_s - d_s||^2 where u_s solves the discrete
Helmholtz problem (L_h(c2) + omega^2) u_s = f_s (eq. discreteHelmholtz) and R
samples receiver nodes.

Face identity for the conservative operator (Section 2.2 discretisation): for
nodal a, b that vanish on the boundary,
    a^T L_h b = -(1/h^2) sum_faces c2_f (a_p - a_q)(b_p - b_q),  c2_f = (c2_p + c2_q)/2,
so d(a^T L_h b)/d c2_k = -(1/(2h^2)) face_sum(a, b)[k] with
face_sum(a, b)[k] = sum over the faces touching node k of (a_k - a_q)(b_k - b_q).

Two independent gradients are provided:
* ``grad_direct``: dJ/dc2 = -sum_s lam_s^T (dL_h/dc2) u_s with
  lam_s = (L_h + omega^2)^{-1} R^T (R u_s - d_s)  (direct sparse solves);
* ``vjp_time_domain``: the fixed point u = Pi_h(u; c2) gives
  dJ/dc2 = (dPi_h/dc2)^T z with z = A^{-1} R^T (R u - d) (A = I - S_h is symmetric);
  the VJP runs the transposed leapfrog recurrence backwards with the filter
  weights as source:  Lam^{N_t} = w_{N_t} z,
  Lam^n = (2 + dt^2 L_h) Lam^{n+1} - Lam^{n+2} + w_n z  (n = N_t-1..1),
  and collects  dt^2 sum_{n>=1} (Lam^{n+1})^T (dL_h/dc2) W^n + dt^2/2 (Lam^1)^T (dL_h/dc2) W^0
  along the forward trajectory W^n of Pi_h(u; f).
"""
from __future__ import annotations

import numpy as np

from . import discretization as disc
from . import wavesolve


def face_sum(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Per node k: sum over its grid faces (k, q) of (a_k - a_q)(b_k - b_q)."""
    out = np.zeros_like(a, dtype=np.float64)
    for ax in range(a.ndim):
        da = np.diff(a, axis=ax)
        db = np.diff(b, axis=ax)
        prod = da * db                      # face between i and i+1 along ax
        lo = [slice(None)] * a.ndim; lo[ax] = slice(0, -1)
        hi = [slice(None)] * a.ndim; hi[ax] = slice(1, None)
        out[tuple(lo)] += prod
        out[tuple(hi)] += prod
    return out


def restrict(u_nodal: np.ndarray, rec_idx) -> np.ndarray:
    return u_nodal.reshape(-1)[rec_idx]


def restrict_T(vals, rec_idx, shape) -> np.ndarray:
    g = np.zeros(int(np.prod(shape)))
    np.add.at(g, rec_idx, vals)
    return g.reshape(shape)


def forward(dim, n, c2, omega, sources, rec_idx):
    L = disc.laplacian(dim, n, c2)
    us = [disc.to_nodal(disc.direct_solve(L, omega, disc.to_interior(f)), dim, n) for f in sources]
    return L, us


def misfit(dim, n, c2, omega, sources, rec_idx, d) -> float:
    _, us = forward(dim, n, c2, omega, sources, rec_idx)
    return 0.5 * sum(float(np.sum((restrict(u, rec_idx) - d[s]) ** 2)) for s, u in enumerate(us))


def grad_direct(dim, n, c2, omega, sources, rec_idx, d):
    """(J, dJ/dc2 on all nodes) by direct solves."""
    h = 1.0 / n
    L, us = forward(dim, n, c2, omega, sources, rec_idx)
    from scipy.sparse.linalg import splu
    lu = splu(disc.helmholtz_matrix(L, omega))
    J = 0.0
    g = np.zeros((n + 1,) * dim)
    for s, u in enumerate(us):
        res = restrict(u, rec_idx) - d[s]
        J += 0.5 * float(res @ res)
        rhs = disc.to_interior(restrict_T(res, rec_idx, u.shape))
        lam = disc.to_nodal(lu.solve(rhs), dim, n)
        g += face_sum(lam, u) / (2.0 * h * h)
    return J, g


def vjp_time_domain(L, dim, n, u_int, z_int, f_int, tp):
    """(dPi_h(u; f)/dc2)^T z on all nodes, by the backward recurrence above."""
    h = 1.0 / n
    traj = []
    wavesolve.wave_filter(L, u_int, f_int, tp, trajectory=traj)
    N = tp.nt
    dt2 = tp.dt ** 2
    lam_next2 = np.zeros_like(z_int)          # Lam^{n+2}
    lam_next = tp.weights[N] * z_int           # Lam^{n+1}, starting at Lam^{N}
    g = np.zeros((n + 1,) * dim)
    for nn in range(N - 1, 0, -1):
        # contribution of step nn (uses Lam^{nn+1} and W^{nn})
        g += -dt2 / (2 * h * h) * face_sum(disc.to_nodal(lam_next, dim, n), disc.to_nodal(traj[nn], dim, n))
        lam = 2.0 * lam_next + dt2 * (L @ lam_next) - lam_next2 + tp.weights[nn] * z_int
        lam_next2, lam_next = lam_next, lam
    # first half step: dt^2/2 (Lam^1)^T dL W^0
    g += -0.5 * dt2 / (2 * h * h) * face_sum(disc.to_nodal(lam_next, dim, n), disc.to_nodal(traj[0], dim, n))
    return g


def fd_directional(dim, n, c2, omega, sources, rec_idx, d, delta, eps=1e-6) -> float:
    """Central difference (J(c2 + eps delta) - J(c2 - eps delta)) / (2 eps)."""
    jp = misfit(dim, n, c2 + eps * delta, omega, sources, rec_idx, d)
    jm = misfit(dim, n, c2 - eps * delta, omega, sources, rec_idx, d)
    return (jp - jm) / (2 * eps)
