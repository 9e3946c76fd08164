"""Pins of the oracle's misfit gradient: central finite differences, and the
agreement of two independent derivations (direct-solve adjoint and the
time-reversed VJP of the filter at the fixed point)."""
import numpy as np
import pytest

import workloads as wl
from oracle import adjoint, discretization as disc, timeparams as tpm, wavesolve as ws, krylov


def _case(n=12, n_src=2, seed=11):
    rng = np.random.default_rng(seed)
    c2 = wl.config5_c2(n, rng)
    c2_ref = wl.config5_c2(n, rng)
    srcs = [wl.gaussian(2, n, rng.uniform(0.2, 0.8, 2), 0.15) for _ in range(n_src)]
    rec = np.array([j * (n + 1) + i for j in (2, n - 2) for i in range(1, n)] +
                   [j * (n + 1) + i for i in (3,) for j in range(1, n)], dtype=np.int64)
    omega = 9.7
    _, us_ref = adjoint.forward(2, n, c2_ref, omega, srcs, rec)
    d = [adjoint.restrict(u, rec) for u in us_ref]
    return n, c2, omega, srcs, rec, d


def test_face_identity():
    n = 9
    rng = np.random.default_rng(0)
    c2 = wl.config5_c2(n, rng)
    L = disc.laplacian(2, n, c2)
    a = wl.random_nodal(2, n, 1); b = wl.random_nodal(2, n, 2)
    lhs = disc.to_interior(a) @ (L @ disc.to_interior(b))
    # a^T L_h b = -(1/h^2) sum_faces c2_f da db; with face_sum counting each face at both nodes,
    # sum_k c2_k face_sum(a,b)[k] = 2 sum_faces c2_f da db
    rhs = -(n * n) * 0.5 * np.sum(c2 * adjoint.face_sum(a, b))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_direct_gradient_matches_central_fd():
    n, c2, omega, srcs, rec, d = _case()
    J, g = adjoint.grad_direct(2, n, c2, omega, srcs, rec, d)
    assert J > 0
    rng = np.random.default_rng(3)
    for _ in range(4):
        delta = rng.standard_normal(c2.shape)
        delta /= np.abs(delta).max()
        fd = adjoint.fd_directional(2, n, c2, omega, srcs, rec, d, delta, eps=1e-6)
        an = float(np.sum(g * delta))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.abs(g).sum())


def test_time_domain_vjp_matches_direct_gradient():
    n, c2, omega, srcs, rec, d = _case(n=10, n_src=2)
    J, g_direct = adjoint.grad_direct(2, n, c2, omega, srcs, rec, d)
    L = disc.laplacian(2, n, c2)
    tp = tpm.time_parameters(omega, 1.0 / n, float(np.sqrt(c2.max())))
    A = ws.dense_A(L, tp)
    g_td = np.zeros_like(c2)
    for s, f in enumerate(srcs):
        fi = disc.to_interior(f)
        u = disc.direct_solve(L, omega, fi)
        res = adjoint.restrict(disc.to_nodal(u, 2, n), rec) - d[s]
        gu = disc.to_interior(adjoint.restrict_T(res, rec, c2.shape))
        z = np.linalg.solve(A, gu)
        g_td += adjoint.vjp_time_domain(L, 2, n, u, z, fi, tp)
    assert np.abs(g_td - g_direct).max() < 1e-8 * np.abs(g_direct).max()


def test_time_domain_vjp_is_independent_of_dt():
    # under the corrected frequency the fixed point (hence J) does not depend on dt
    n, c2, omega, srcs, rec, d = _case(n=10, n_src=1)
    L = disc.laplacian(2, n, c2)
    fi = disc.to_interior(srcs[0])
    u = disc.direct_solve(L, omega, fi)
    res = adjoint.restrict(disc.to_nodal(u, 2, n), rec) - d[0]
    gu = disc.to_interior(adjoint.restrict_T(res, rec, c2.shape))
    out = []
    for cfl in (0.5, 0.3):
        tp = tpm.time_parameters(omega, 1.0 / n, float(np.sqrt(c2.max())), cfl=cfl)
        A = ws.dense_A(L, tp)
        z = np.linalg.solve(A, gu)
        out.append(adjoint.vjp_time_domain(L, 2, n, u, z, fi, tp))
    assert np.abs(out[0] - out[1]).max() < 1e-8 * np.abs(out[0]).max()
