"""Small seeded cases shared by the CPU oracle tests."""
import numpy as np

import workloads as wl
from oracle import discretization as disc, timeparams as tpm


def setup(dim, n, omega, c2=None, f=None, cfl=0.5, n_periods=1, seed=0, **kw):
    L = disc.laplacian(dim, n, c2)
    cmax = 1.0 if c2 is None else float(np.sqrt(np.max(c2)))
    tp = tpm.time_parameters(omega, 1.0 / n, cmax, cfl=cfl, n_periods=n_periods, **kw)
    if f is None:
        f = wl.gaussian(dim, n, (0.43, 0.55, 0.5)[:dim], 0.1)
    return L, tp, disc.to_interior(f)


def varc2(dim, n, seed=7, amp=0.3):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-amp, amp, size=4)
    xs = rng.uniform(0.2, 0.8, size=(4, dim))
    c = 1.0 + wl.gaussian_sum_field(dim, n, a, xs, 0.15)
    return c * c
