"""Second-order finite differences for L = div(c^2 grad) on the unit box.

Follows Section 2.2 (eq. discreteHelmholtz): grid points x_j = j h,
j = 0..n, h = 1/n, with the interior equation on j = 1..n-1 and the Dirichlet
condition W = 0 on the boundary nodes (eq. helmholtzBVP, operator eq. L).

The variable-coefficient operator is the conservative 2d+1-point form
    (L_h W)_p = (1/h^2) sum_{faces (p,q)} c2_f (W_q - W_p),
    c2_f = (c2_p + c2_q)/2,
which is symmetric; with c2 = 1 it is the standard 5-/7-point Laplacian.

Fourth order (the paper's spatial order; c = 1 only here): per axis the centred
difference h^-2 (-W_{i-2} + 16 W_{i-1} - 30 W_i + 16 W_{i+1} - W_{i+2}) / 12, with the
Dirichlet boundary closed by odd reflection, W_{-1} = -W_1 and W_{n+1} = -W_{n-1}
(the compatibility W_xx = 0 of a boundary where W and f vanish).  The first interior
row becomes (-29 W_1 + 16 W_2 - W_3) / 12; the matrix stays symmetric and the sine
vectors stay its eigenvectors, with lam2 = h^-2 (30 - 32 cos t + 2 cos 2t) / 12 per
axis, t = k pi h.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def to_interior(a: np.ndarray) -> np.ndarray:
    """Nodal array (n+1,)*dim -> flat interior vector (x fastest)."""
    return np.ascontiguousarray(a[(slice(1, -1),) * a.ndim]).reshape(-1)


def to_nodal(v: np.ndarray, dim: int, n: int) -> np.ndarray:
    """Flat interior vector -> nodal array with a zero boundary ring."""
    a = np.zeros((n + 1,) * dim, dtype=v.dtype)
    a[(slice(1, -1),) * dim] = v.reshape((n - 1,) * dim)
    return a


def laplacian4_1d(n: int) -> sp.csr_matrix:
    """The fourth-order 1D operator on the n-1 interior nodes (odd reflection at the ends)."""
    h = 1.0 / n
    m = n - 1
    main = np.full(m, -30.0)
    main[0] += 1.0      # W_{-1} = -W_1 folds -(-W_1) into the diagonal
    main[-1] += 1.0
    D = sp.diags([np.full(m - 2, -1.0), np.full(m - 1, 16.0), main, np.full(m - 1, 16.0),
                  np.full(m - 2, -1.0)], [-2, -1, 0, 1, 2], format="csr")
    return D / (12.0 * h * h)


def laplacian(dim: int, n: int, c2: np.ndarray | None = None, order: int = 2) -> sp.csr_matrix:
    """L_h as a sparse matrix on the interior unknowns."""
    if order == 4:
        assert c2 is None, "fourth order is built for c = 1"
        D = laplacian4_1d(n)
        I = sp.identity(n - 1, format="csr")
        if dim == 2:
            return (sp.kron(I, D) + sp.kron(D, I)).tocsr()          # x fastest
        return (sp.kron(sp.kron(I, I), D) + sp.kron(sp.kron(I, D), I) + sp.kron(sp.kron(D, I), I)).tocsr()
    assert order == 2
    h = 1.0 / n
    shape = (n + 1,) * dim
    if c2 is None:
        c2 = np.ones(shape)
    c2 = np.asarray(c2, dtype=np.float64)
    assert c2.shape == shape
    # interior numbering, -1 on the boundary
    idx = -np.ones(shape, dtype=np.int64)
    idx[(slice(1, -1),) * dim] = np.arange((n - 1) ** dim).reshape((n - 1,) * dim)
    inner = (slice(1, -1),) * dim
    p_idx = idx[inner].ravel()
    c2p = c2[inner].ravel()
    rows, cols, vals = [], [], []
    diag = np.zeros(p_idx.size)
    for ax in range(dim):
        for s in (-1, 1):
            nb = list(inner)
            nb[ax] = slice(1 + s, n + s)
            q_idx = idx[tuple(nb)].ravel()
            cf = 0.5 * (c2p + c2[tuple(nb)].ravel()) / h ** 2
            diag -= cf
            m = q_idx >= 0
            rows.append(p_idx[m]); cols.append(q_idx[m]); vals.append(cf[m])
    rows.append(p_idx); cols.append(p_idx); vals.append(diag)
    N = p_idx.size
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def helmholtz_matrix(L: sp.spmatrix, omega: float) -> sp.csc_matrix:
    """L_h + omega^2 I  (eq. discreteHelmholtz)."""
    return (L + omega ** 2 * sp.identity(L.shape[0], format="csr")).tocsc()


def direct_solve(L: sp.spmatrix, omega: float, f: np.ndarray) -> np.ndarray:
    """U* = (L_h + omega^2)^{-1} f by sparse LU: the discrete Helmholtz solution
    that the WaveHoltz fixed point equals (Sections 2.1-2.2)."""
    return spla.splu(helmholtz_matrix(L, omega)).solve(np.asarray(f, dtype=np.float64))


def helmholtz_residual(L, omega, U, f) -> float:
    """||f - (L_h + omega^2) U|| / ||f|| (eq. discreteHelmholtz), interior vectors."""
    r = f - (L @ U + omega ** 2 * U)
    return float(np.linalg.norm(r) / np.linalg.norm(f))


def direct_solve_dst(dim: int, n: int, omega: float, f_nodal: np.ndarray, order: int = 2) -> np.ndarray:
    """U* for c = 1 by diagonalising L_h with the type-I discrete sine transform:
    L_h = -S diag(lam2) S with the orthonormal sine basis S (eq. discreteEigenvalueProblem;
    lam2 = (4/h^2) sum_axes sin^2(k pi h/2)), so U = S diag(1/(omega^2 - lam2)) S f.
    Exact up to rounding; returns the nodal solution."""
    from scipy.fft import dstn, idstn
    h = 1.0 / n
    k = np.arange(1, n)
    if order == 4:
        t = k * np.pi * h
        e1 = (30.0 - 32.0 * np.cos(t) + 2.0 * np.cos(2.0 * t)) / (12.0 * h * h)
    else:
        e1 = (4.0 / h ** 2) * np.sin(k * np.pi * h / 2.0) ** 2
    lam2 = sum(np.meshgrid(*([e1] * dim), indexing="ij"))
    fi = np.asarray(f_nodal, dtype=np.float64)[(slice(1, -1),) * dim]
    fh = dstn(fi, type=1, norm="ortho")
    U = idstn(fh / (omega ** 2 - lam2), type=1, norm="ortho")
    out = np.zeros((n + 1,) * dim)
    out[(slice(1, -1),) * dim] = U
    return out
