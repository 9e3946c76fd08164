"""Seeded synthetic inputs for the WaveHoltz Helmholtz workloads.

This module only *draws* inputs: grids, wave speeds, sources, frequencies,
receiver positions and perturbation directions.  It holds none of the
solver's arithmetic (no time stepping, no filter, no Krylov method) and is
the one module shared by the CPU oracle and by the GPU path's tests and
benchmark.  Every array is nodal: shape ``(n+1,)*dim`` with the last axis
being x, node ``i`` at coordinate ``i*h`` with ``h = 1/n`` (unit box,
homogeneous Dirichlet, so boundary entries of sources are set to zero).

Gaussian source shapes follow the paper's time-harmonic Gaussian source
(Section 5, eq. gaussianSource): ``a * exp(-b^2 |x-x0|^2)``; where a
workload states a width ``w`` the exponent is ``|x-x0|^2 / w^2``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def coords(dim: int, n: int):
    """Nodal coordinate arrays (z, y, x order for 3D; y, x for 2D)."""
    x = np.arange(n + 1, dtype=np.float64) / n
    return np.meshgrid(*([x] * dim), indexing="ij")


def zero_boundary(a: np.ndarray) -> np.ndarray:
    a = a.copy()
    for ax in range(a.ndim):
        sl = [slice(None)] * a.ndim
        sl[ax] = 0
        a[tuple(sl)] = 0.0
        sl[ax] = -1
        a[tuple(sl)] = 0.0
    return a


def gaussian(dim: int, n: int, center, width: float, amplitude: float = 1.0) -> np.ndarray:
    """amplitude * exp(-|x - center|^2 / width^2) on the nodes, zero on the boundary."""
    X = coords(dim, n)
    # X is ordered (z, y, x) / (y, x); center is given as (x, y[, z])
    c = list(center)[::-1]
    r2 = sum((X[k] - c[k]) ** 2 for k in range(dim))
    return zero_boundary(amplitude * np.exp(-r2 / width ** 2))


def gaussian_sum_field(dim: int, n: int, amps, centers, width: float) -> np.ndarray:
    """sum_i amps[i] * exp(-|x - centers[i]|^2 / width^2) on all nodes (boundary included)."""
    X = coords(dim, n)
    P = np.zeros((n + 1,) * dim)
    for a, c in zip(amps, centers):
        cc = list(c)[::-1]
        P += a * np.exp(-sum((X[k] - cc[k]) ** 2 for k in range(dim)) / width ** 2)
    return P


@dataclass
class Problem:
    """One Helmholtz problem  L u + omega^2 u = f  on the unit box."""
    dim: int
    n: int
    omega: float
    f: np.ndarray                      # nodal source, zero boundary
    c2: Optional[np.ndarray] = None    # nodal c^2 incl. boundary; None means c = 1
    name: str = ""
    meta: dict = field(default_factory=dict)


# ---------------------------------------------------------------- config 1
def config1(n: int = 64) -> Problem:
    """2D unit square, c=1, omega=20.5, f=exp(-((x-.5)^2+(y-.5)^2)/0.05^2)."""
    return Problem(2, n, 20.5, gaussian(2, n, (0.5, 0.5), 0.05), None, "cfg1-2d-64-cg-f64")


# ---------------------------------------------------------------- config 2
def config2(n: int = 1024, omega: float = 100.3, seed: int = 2) -> Problem:
    """2D unit square, c=1, Gaussian of width 0.02 at a seeded centre in [.2,.8]^2."""
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0.2, 0.8, size=2)
    return Problem(2, n, omega, gaussian(2, n, x0, 0.02), None, f"cfg2-2d-{n}-dcg32",
                   {"x0": x0.tolist(), "n_defl": 32})


# ---------------------------------------------------------------- config 3
def config3_c(n: int = 256, seed: int = 3) -> np.ndarray:
    """c(x) = 1 + sum_{i<8} a_i exp(-|x-x_i|^2/0.1^2); returns nodal c^2 (= c*c)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-0.3, 0.3, size=8)
    xs = rng.uniform(0.2, 0.8, size=(8, 3))
    c = 1.0 + gaussian_sum_field(3, n, a, xs, 0.1)
    return c * c


def config3(n: int = 256, omega: float = 40.0, seed: int = 3) -> Problem:
    c2 = config3_c(n, seed)
    f = gaussian(3, n, (0.5, 0.5, 0.5), 0.05)
    return Problem(3, n, omega, f, c2, f"cfg3-3d-{n}-varc")


# ---------------------------------------------------------------- config 4
def dirichlet_5pt_eigs_sqrt(n: int, lam_max: float) -> np.ndarray:
    """Sorted square roots of the eigenvalues of the negative 5-point Dirichlet
    Laplacian on the unit square (textbook closed form), up to lam_max.

    Used only as an input-admissibility filter (keeping drawn frequencies away
    from resonance); it is not a step of any solver.
    """
    h = 1.0 / n
    k = np.arange(1, n)
    s = (4.0 / h ** 2) * np.sin(k * np.pi * h / 2) ** 2
    s = s[s <= lam_max ** 2]
    lam = np.sqrt(s[:, None] + s[None, :]).ravel()
    return np.sort(lam[lam <= lam_max])


def gap_ok(n: int, omega: float, rel: float = 0.01) -> bool:
    """Accept omega iff its distance to the nearest discrete eigenvalue is at least
    ``rel`` times the spacing of the two eigenvalues that bracket it."""
    lam = dirichlet_5pt_eigs_sqrt(n, 2.0 * omega + 10.0)
    i = np.searchsorted(lam, omega)
    if i == 0 or i >= len(lam):
        return True
    lo, hi = lam[i - 1], lam[i]
    return min(omega - lo, hi - omega) >= rel * (hi - lo)


def config4(sizes=(128, 256, 512, 1024), per_size: int = 64, seed: int = 4,
            omega_range=(10.0, 80.0)) -> List[Problem]:
    """Batched workload: ``per_size`` problems on each grid size, omega~U(10,80)
    redrawn until it clears the resonance-gap rule, source omega^2 exp(-omega^2 r^2)."""
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        for k in range(per_size):
            while True:
                om = float(rng.uniform(*omega_range))
                if gap_ok(n, om):
                    break
            x0 = rng.uniform(0.2, 0.8, size=2)
            f = gaussian(2, n, x0, 1.0 / om, amplitude=om * om)
            out.append(Problem(2, n, om, f, None, f"cfg4-{n}-{k}", {"x0": x0.tolist()}))
    return out


# ---------------------------------------------------------------- N_D sweep
def ppw_grid_points(omega: float, order: int = 2, eps: float = 1e-3, size: float = 1.0,
                    c: float = 1.0) -> float:
    """Grid points per direction from the points-per-wavelength rule of thumb for an
    order-p scheme (Section 2.2, eq. NxFromPPW): N = w (w b / (2 eps))^(1/p) with the
    non-dimensional frequency w = omega size / c and b = 2 (q!)^2 / (2q+2)!, q = p/2."""
    q = order // 2
    b = 2.0 * math.factorial(q) ** 2 / math.factorial(2 * q + 2)
    wn = omega * size / c
    return wn * (wn * b / (2.0 * eps)) ** (1.0 / order)


def ndsweep_problem(omega: float, eps: float = 1e-3) -> Problem:
    """The frequency sweep of the deflation-size study (Section 4.2) on the unit square
    with c = 1 and the second-order scheme: n from the PPW rule with relative error eps,
    source omega^2 exp(-omega^2 |x - x0|^2) (eq. gaussianSource with a = omega^2,
    b = omega) at the fixed interior point x0 = (0.3, 0.4)."""
    n = int(math.ceil(ppw_grid_points(omega, 2, eps)))
    f = gaussian(2, n, (0.3, 0.4), 1.0 / omega, amplitude=omega * omega)
    return Problem(2, n, float(omega), f, None, f"ndsweep-{omega:g}", {"eps": eps})


# ---------------------------------------------------------------- config 5
def config5_c2(n: int, rng) -> np.ndarray:
    """c^2 = 1 + 0.2 P / max|P|, P a sum of 8 Gaussians (width 0.1) with a_i~U(-1,1)."""
    a = rng.uniform(-1.0, 1.0, size=8)
    xs = rng.uniform(0.2, 0.8, size=(8, 2))
    P = gaussian_sum_field(2, n, a, xs, 0.1)
    return 1.0 + 0.2 * P / np.max(np.abs(P))


def receivers(n: int, per_line: int = 128) -> np.ndarray:
    """Nodal linear indices (row-major, x fastest) of receivers on the four grid
    lines x=n/8, x=7n/8, y=n/8, y=7n/8, at every (n/per_line)-th node (offset half a stride)."""
    stride = n // per_line
    pos = stride * np.arange(1, per_line + 1) - stride // 2
    a, b = n // 8, (7 * n) // 8
    idx = []
    for xl in (a, b):           # vertical lines x = const: nodes (j=pos, i=xl)
        idx += [int(j) * (n + 1) + xl for j in pos]
    for yl in (a, b):           # horizontal lines y = const
        idx += [yl * (n + 1) + int(i) for i in pos]
    return np.asarray(idx, dtype=np.int64)


@dataclass
class AdjointWorkload:
    n: int
    omega: float
    c2: np.ndarray
    c2_ref: np.ndarray
    sources: List[np.ndarray]
    rec_idx: np.ndarray
    c_max: float
    directions: np.ndarray   # (n_dir, n+1, n+1), sup-norm 1


def config5(n: int = 512, n_src: int = 16, omega: float = 30.0, seed: int = 5,
            per_line: int = 128, n_dir: int = 20) -> AdjointWorkload:
    rng = np.random.default_rng(seed)
    c2 = config5_c2(n, rng)
    c2_ref = config5_c2(n, rng)
    srcs = []
    for _ in range(n_src):
        x0 = rng.uniform(0.15, 0.85, size=2)
        srcs.append(gaussian(2, n, x0, 0.01))
    dirs = rng.standard_normal((n_dir, n + 1, n + 1))
    dirs /= np.max(np.abs(dirs), axis=(1, 2), keepdims=True)
    return AdjointWorkload(n, omega, c2, c2_ref, srcs, receivers(n, min(per_line, n // 2)),
                           math.sqrt(1.2), dirs)


def random_nodal(dim: int, n: int, seed: int) -> np.ndarray:
    """Seeded standard-normal nodal field with a zero boundary ring."""
    rng = np.random.default_rng(seed)
    return zero_boundary(rng.standard_normal((n + 1,) * dim))
