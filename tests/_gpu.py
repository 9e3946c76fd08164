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


def oracle_tp(dim, n, omega, c2=None, **kw):
    cmax = 1.0 if c2 is None else float(np.sqrt(np.max(c2)))
    return tpm.time_parameters(omega, 1.0 / n, cmax, **kw)


def direct(dim, n, omega, f, c2=None):
    L = disc.laplacian(dim, n, c2)
    return disc.to_nodal(disc.direct_solve(L, omega, disc.to_interior(f)), dim, n)
