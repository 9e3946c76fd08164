"""Direct eigenvector deflation (DEVD), Algorithm 2 in discrete form.

With orthonormal discrete eigenvectors phi_m (L_h phi_m = -lam2_m phi_m):
  1. deflate the forcing:  f_d = f - sum_m (f, phi_m) phi_m;
  2. solve the WaveHoltz problem for f_d (FPI or CG), optionally deflating each
     iterate (v <- v - sum_m (v, phi_m) phi_m);
  3. inflate:  u = v + sum_m (f, phi_m) / (omega^2 - lam2_m) phi_m.
(f, phi) is the l2 inner product over interior nodes.  The inflation uses the
Helmholtz omega and the discrete lam2, which is exact for the fixed point of the
time-corrected scheme (it solves L_h + omega^2 exactly).
"""
from __future__ import annotations

import numpy as np

from . import krylov, wavesolve


def deflate(W, v):
    return v - W @ (W.T @ v)


def inflate(W, lam2, omega, f, v):
    return v + W @ ((W.T @ f) / (omega ** 2 - np.asarray(lam2)))


def devd_solve(L, f, tp, W, lam2, method="cg", tol=1e-10, maxit=10000, deflate_iterates=False):
    fd = deflate(W, f)
    b = wavesolve.rhs(L, fd, tp)
    if method == "cg":
        v, info = krylov.cg(lambda x: wavesolve.apply_A(L, x, tp), b, tol=tol, maxit=maxit)
    elif method == "fpi":
        def Pi(x):
            y = wavesolve.wave_filter(L, x, fd, tp)
            return deflate(W, y) if deflate_iterates else y
        v, info = krylov.fpi(Pi, b, tol=tol, maxit=maxit)
    else:
        raise ValueError(method)
    return inflate(W, lam2, tp.omega, f, v), info
