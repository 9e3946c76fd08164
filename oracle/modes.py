"""Analytic Dirichlet eigenvectors of the constant-coefficient Laplacian.

On the unit box with n cells, the 5-/7-point operator L_h (c = 1) has the
tensor-product eigenvectors (Section 4.4: the one-dimensional vectors
z_{k,i} = d_k sin(pi k (r_i+1)/2) on [-1,1], here mapped to [0,1]):

    Phi_{p,q}(x_i, y_j) = (2/n) sin(p pi x_i) sin(q pi y_j),   p, q = 1..n-1,

l2-orthonormal over the interior nodes (sum_i sin^2(p pi i/n) = n/2), with
    L_h Phi = -lam2 Phi,  lam2 = (4/h^2) sum_axes sin^2(k_axis pi h / 2)
(eq. discreteEigenvalueProblem).  In 3D the factor is (2/n)^{3/2}.

The deflation set takes the N_D modes whose lam2 lie nearest omega^2, the
Helmholtz resonance (Section 2.3 asks for the eigenvectors whose eigenvalues are
closest to the frequency).  Distances are compared on a grid of 1e-9 omega^2, so
that modes whose lam2 agree up to rounding (degenerate mode sets, summed in
different orders) count as ties; ties are broken by the mode index tuple in
lexicographic order.
"""
from __future__ import annotations

import numpy as np


def eig1d(n: int, order: int = 2) -> np.ndarray:
    """lam2 of the 1D operator for k = 1..n-1 (index k-1); order 4: the fourth-order
    difference with odd reflection at the ends (the sine vectors are its eigenvectors)."""
    h = 1.0 / n
    k = np.arange(1, n)
    if order == 4:
        t = k * np.pi * h
        return (30.0 - 32.0 * np.cos(t) + 2.0 * np.cos(2.0 * t)) / (12.0 * h * h)
    return (4.0 / h ** 2) * np.sin(k * np.pi * h / 2.0) ** 2


def mode_lam2(dim: int, n: int, idx, order: int = 2) -> float:
    e = eig1d(n, order)
    return float(sum(e[k - 1] for k in idx))


def select_modes(dim: int, n: int, omega: float, n_defl: int, order: int = 2):
    """The n_defl mode index tuples (x index first) nearest to resonance."""
    e = eig1d(n, order)
    ks = np.arange(1, n)
    if dim == 2:
        P, Q = np.meshgrid(ks, ks, indexing="ij")
        lam2 = e[P - 1] + e[Q - 1]
        tuples = np.stack([P.ravel(), Q.ravel()], axis=1)
    else:
        P, Q, R = np.meshgrid(ks, ks, ks, indexing="ij")
        lam2 = e[P - 1] + e[Q - 1] + e[R - 1]
        tuples = np.stack([P.ravel(), Q.ravel(), R.ravel()], axis=1)
    dist = np.abs(lam2.ravel() - omega ** 2)
    # distances on a grid of 1e-9 omega^2, then lexicographic tie-break: (dist, p, q[, r])
    dq = np.floor(dist / (1e-9 * omega ** 2) + 0.5)
    keys = [tuples[:, k] for k in range(dim - 1, -1, -1)] + [dq]
    order = np.lexsort(keys)[:n_defl]
    return [tuple(int(v) for v in tuples[i]) for i in order], lam2.ravel()[order]


def mode_nodal(dim: int, n: int, idx) -> np.ndarray:
    """Phi_idx on the nodal grid (zero on the boundary); idx is (p_x, q_y[, r_z])."""
    x = np.arange(n + 1) / n
    norm = np.sqrt(2.0 / n)
    s = [norm * np.sin(k * np.pi * x) for k in idx]
    if dim == 2:
        a = np.outer(s[1], s[0])               # [j (y), i (x)]
    else:
        a = np.einsum("k,j,i->kji", s[2], s[1], s[0])
    # exact zeros on the boundary
    for ax in range(dim):
        sl = [slice(None)] * dim
        sl[ax] = 0; a[tuple(sl)] = 0.0
        sl[ax] = -1; a[tuple(sl)] = 0.0
    return a


def mode_matrix(dim: int, n: int, modes) -> np.ndarray:
    """W in R^{N x N_D}: columns are the interior values of the modes."""
    inner = (slice(1, -1),) * dim
    return np.stack([mode_nodal(dim, n, m)[inner].ravel() for m in modes], axis=1)
