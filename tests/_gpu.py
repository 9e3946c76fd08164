"""Helpers for the GPU parity tests (oracle on the CPU, library on the GPU)."""
import numpy as np

from oracle import discretization as disc, timeparams as tpm


def cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def relmx(a, b):
    """The larger of the 2-norm relative error and the element-wise one (relative to max |b|)."""
    return max(rel(a, b), maxrel(a, b))


def maxrel(a, b):
    """Element-wise: max_i |a_i - b_i| / max_i |b_i|."""
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def assert_close(got, want, tol, what=""):
    """Both the 2-norm relative error and the element-wise error (relative to max |want|) <= tol."""
    e2, em = rel(got, want), maxrel(got, want)
    print(f"  {what} err 2-norm {e2:.2e} max {em:.2e} (bar {tol:.0e})", flush=True)
    assert e2 <= tol and em <= tol, (what, e2, em)


def oracle_tp(dim, n, omega, c2=None, **kw):
    cmax = 1.0 if c2 is None else float(np.sqrt(np.max(c2)))
    return tpm.time_parameters(omega, 1.0 / n, cmax, **kw)


def direct(dim, n, omega, f, c2=None):
    L = disc.laplacian(dim, n, c2)
    return disc.to_nodal(disc.direct_solve(L, omega, disc.to_interior(f)), dim, n)
