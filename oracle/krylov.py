"""Iterative solvers for A x = b with A = I - S_h applied by wave solves (Section 3).

Every solver takes ``A`` as a callable (one call = one wave solve) and stops on
||r||_2 / ||b||_2 <= tol.  Each returns (x, info) with info["iters"] (solver
iterations), info["matvecs"] (applications of A) and info["res"] (the relative
residual history the solver itself tracks).

fpi        WaveHoltz fixed-point iteration, Algorithm 1 (v <- Pi_h v).
cg         conjugate gradients (Algorithm 3 with an empty deflation matrix).
           Breakdown is p^T A p = 0 (or non-finite) only: with the corrected
           frequency A can have a few tiny negative eigenvalues (beta_h peaks at
           1 + O(dt^4) just below omega), and CG still runs on such a system.
dcg        deflated CG of Saad et al., Algorithm 3.  Readings of garbled lines:
           r_2 is r_0^T r_0 on entry; r_{k+1} = r_k - alpha_k q_k; the
           deflated start uses W (W^T A W)^{-1} W^T r_{-1}.
agmres     augmented GMRES with Givens rotations, Algorithm 4, restarted.
           With N_D = 0 it is plain restarted GMRES(m).  Reading of the garbled
           RHS update: g(k+1) = -s g(k), then g(k) = c g(k).
abicgstab  augmented (recycled) BiCGStab, Algorithm 5.
"""
from __future__ import annotations

import numpy as np


def _rel(r, nb):
    return float(np.linalg.norm(r) / nb)


def fpi(Pi, b, v0=None, tol=1e-8, maxit=1000):
    """Algorithm 1: v^{k+1} = Pi_h v^k.  The update v^{k+1}-v^k equals the residual
    b - A v^k, so the stopping test is on that update."""
    nb = np.linalg.norm(b)
    v = np.zeros_like(b) if v0 is None else np.array(v0, dtype=np.float64)
    hist = []
    k = 0
    while k < maxit:
        vn = Pi(v)
        k += 1
        hist.append(_rel(vn - v, nb))
        v = vn
        if hist[-1] <= tol:
            break
    return v, {"iters": k, "matvecs": k, "res": hist}


def cg(A, b, x0=None, tol=1e-10, maxit=10000):
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A(x) if x0 is not None else b.copy()
    mv = 1 if x0 is not None else 0
    p = r.copy()
    r2 = float(r @ r)
    hist = [np.sqrt(r2) / nb]
    k = 0
    while hist[-1] > tol and k < maxit:
        q = A(p); mv += 1
        pq = float(p @ q)
        if pq == 0 or not np.isfinite(pq):
            raise FloatingPointError("CG breakdown: p^T A p = 0")
        alpha = r2 / pq
        x += alpha * p
        r -= alpha * q
        r2n = float(r @ r)
        p = r + (r2n / r2) * p
        r2 = r2n
        k += 1
        hist.append(np.sqrt(r2) / nb)
    return x, {"iters": k, "matvecs": mv, "res": hist}


def dcg(A, b, W, AW, tol=1e-10, maxit=10000, x_init=None, reproject=True):
    """Algorithm 3.  ``AW`` = A W (for exact eigenvectors W diag(mu), no wave solve).
    ``reproject=False`` drops the per-iteration A-orthogonalisation against W
    (allowed with exact eigenvectors)."""
    nb = np.linalg.norm(b)
    WtAW = W.T @ AW
    solve_small = lambda y: np.linalg.solve(WtAW, y)
    xm = np.zeros_like(b) if x_init is None else np.array(x_init, dtype=np.float64)
    mv = 0
    if x_init is None:
        rm = b.copy()
    else:
        rm = b - A(xm); mv += 1
    x = xm + W @ solve_small(W.T @ rm)
    r = b - A(x); mv += 1
    # eta_0 = W^T A r_0 = (A W)^T r_0 since A is symmetric
    mu = solve_small(AW.T @ r)
    p = r - W @ mu
    r2 = float(r @ r)
    hist = [np.sqrt(r2) / nb]
    wtr = [float(np.max(np.abs(W.T @ r)))]
    k = 0
    while hist[-1] > tol and k < maxit:
        q = A(p); mv += 1
        pq = float(p @ q)
        if pq == 0 or not np.isfinite(pq):
            raise FloatingPointError("DCG breakdown: p^T A p = 0")
        alpha = r2 / pq
        x += alpha * p
        r -= alpha * q
        r2n = float(r @ r)
        beta = r2n / r2
        r2 = r2n
        if reproject:
            mu = solve_small(AW.T @ r)
            p = beta * p + r - W @ mu
        else:
            p = beta * p + r
        k += 1
        hist.append(np.sqrt(r2) / nb)
        wtr.append(float(np.max(np.abs(W.T @ r))))
    return x, {"iters": k, "matvecs": mv, "res": hist, "wtr": wtr}


def _givens(a, b):
    d = np.hypot(a, b)
    return (1.0, 0.0, 0.0) if d == 0 else (a / d, b / d, d)


def agmres(A, b, x0=None, W=None, AW=None, restart=40, tol=1e-8, maxit=1000):
    """Algorithm 4, restarted every ``restart`` Arnoldi steps.  Stops on
    |g(k+1)| < tol ||b|| (the Givens-updated least-squares residual, which equals
    ||b - A x_k|| in exact arithmetic)."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    nd = 0 if W is None else W.shape[1]
    if nd:
        # reduced QR of A W: A W = V_{1:N_D} H_{1:N_D,1:N_D}
        Qw, Rw = np.linalg.qr(AW)
    mv = 0
    its = 0
    hist = []
    gres = []
    while True:
        b0 = b - A(x) if (its > 0 or x0 is not None) else b.copy()
        if its > 0 or x0 is not None:
            mv += 1
        hist.append(_rel(b0, nb))
        if hist[-1] <= tol or its >= maxit:
            break
        m = restart
        V = np.zeros((b.size, nd + m + 1))
        H = np.zeros((nd + m + 1, nd + m))
        g = np.zeros(nd + m + 1)
        cs = np.zeros(nd + m)
        sn = np.zeros(nd + m)
        v = b0.copy()
        if nd:
            V[:, :nd] = Qw
            H[:nd, :nd] = Rw
            v = v - Qw @ (Qw.T @ v)
        beta0 = np.linalg.norm(v)
        V[:, nd] = v / beta0
        for k in range(nd + 1):
            g[k] = V[:, k] @ b0
        kk = nd
        done = False
        for k in range(nd, nd + m):
            w = A(V[:, k]); mv += 1
            for i in range(k + 1):                  # modified Gram-Schmidt
                H[i, k] = V[:, i] @ w
                w = w - H[i, k] * V[:, i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0:
                V[:, k + 1] = w / H[k + 1, k]
            for i in range(nd, k):                  # previous rotations on the new column
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            c, s, d = _givens(H[k, k], H[k + 1, k])
            cs[k], sn[k] = c, s
            H[k, k] = d
            H[k + 1, k] = 0.0
            g[k + 1] = -s * g[k]
            g[k] = c * g[k]
            its += 1
            kk = k + 1
            gres.append(abs(g[k + 1]) / nb)
            if abs(g[k + 1]) < tol * nb or its >= maxit or H[k, k] == 0:
                done = True
                break
        y = np.linalg.solve(np.triu(H[:kk, :kk]), g[:kk])
        basis = np.concatenate([W, V[:, nd:kk]], axis=1) if nd else V[:, :kk]
        x = x + basis @ y
        if done and (abs(g[kk]) < tol * nb or its >= maxit):
            b0 = b - A(x); mv += 1
            hist.append(_rel(b0, nb))
            break
    return x, {"iters": its, "matvecs": mv, "res": hist, "gres": gres}


def abicgstab(A, b, x0=None, W=None, AW=None, tol=1e-8, maxit=1000):
    """Algorithm 5 (augmented / recycled BiCGStab).  With W = None it is BiCGStab.
    The projection uses Q from the thin QR  A W = Q R; the W-part of the solution
    is recovered at the end as  x -= W R^{-1} xi."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A(x) if x0 is not None else b.copy()
    mv = 1 if x0 is not None else 0
    nd = 0 if W is None else W.shape[1]
    if nd:
        Q, R = np.linalg.qr(AW)
        eta1 = Q.T @ r
        r = r - Q @ eta1
        xi = -eta1
    rt = r.copy()
    hist = [_rel(r, nb)]
    rho_old = alpha = om = 1.0
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    k = 0
    while hist[-1] > tol and k < maxit:
        rho = float(rt @ r)
        if rho == 0:
            break
        if k == 0:
            p = r.copy()
        else:
            beta = (rho / rho_old) * (alpha / om)
            p = r + beta * (p - om * v)
        v = A(p); mv += 1
        if nd:
            e1 = Q.T @ v
            v = v - Q @ e1
        alpha = rho / float(rt @ v)
        s = r - alpha * v
        if np.linalg.norm(s) <= tol * nb:
            x = x + alpha * p
            r = s
            if nd:
                xi = xi + alpha * e1
            k += 1
            hist.append(_rel(r, nb))
            break
        t = A(s); mv += 1
        if nd:
            e2 = Q.T @ t
            t = t - Q @ e2
        om = float(t @ s) / float(t @ t)
        if nd:
            xi = xi + alpha * e1 + om * e2
        x = x + alpha * p + om * s
        r = s - om * t
        rho_old = rho
        k += 1
        hist.append(_rel(r, nb))
    if nd:
        x = x - W @ np.linalg.solve(R, xi)
    return x, {"iters": k, "matvecs": mv, "res": hist}
