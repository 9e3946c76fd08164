"""Preprocessing for factored deflation sets (WH_DEFL_FACTORED): the compression of
Section 4.3, run once on the host before any solve and not part of the library.

Each 2D nodal eigenvector V[k] of L_h ((n+1) x (n+1), y rows, x columns) is replaced by
its truncated singular value decomposition, keeping the singular values above tol times
the largest; term t of the result is the separable product fy[t](y) fx[t](x) with the
singular value folded into fy, and term_mode[t] names the eigenvector it belongs to
(non-decreasing).  The library applies W and W^T from these factors
(paper_2606_31842_amd.factored_deflation).

As a program:
    python compress_modes.py MODES.npy OUT.npz [--tol 1e-5]
reads a float64 array of shape (n_d, n+1, n+1) and writes fx, fy, term_mode and ranks."""
from __future__ import annotations

import argparse

import numpy as np


def compress_modes(V, tol: float = 1e-5):
    """(fx, fy, term_mode, ranks) of the nodal modes V (n_d, n+1, n+1) at the relative
    singular-value cut-off tol (Section 4.3)."""
    V = np.asarray(V, dtype=np.float64)
    if V.ndim != 3 or V.shape[1] != V.shape[2]:
        raise ValueError("V must have shape (n_d, n+1, n+1)")
    fxs, fys, tm, ranks = [], [], [], []
    for k in range(V.shape[0]):
        U, sv, Vt = np.linalg.svd(V[k])
        r = max(1, int(np.sum(sv > tol * sv[0])))
        ranks.append(r)
        for j in range(r):
            fys.append(U[:, j] * sv[j])
            fxs.append(Vt[j])
            tm.append(k)
    return np.array(fxs), np.array(fys), np.array(tm, dtype=np.int32), np.array(ranks)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("modes", help=".npy file, float64 (n_d, n+1, n+1)")
    ap.add_argument("out", help=".npz file to write (fx, fy, term_mode, ranks)")
    ap.add_argument("--tol", type=float, default=1e-5, help="relative singular-value cut-off")
    a = ap.parse_args(argv)
    V = np.load(a.modes, allow_pickle=False)
    fx, fy, tm, ranks = compress_modes(V, a.tol)
    np.savez(a.out, fx=fx, fy=fy, term_mode=tm, ranks=ranks)
    print(f"{V.shape[0]} modes -> {len(tm)} separable terms (ranks {ranks.tolist()})")


if __name__ == "__main__":
    main()
