"""GPU parity of deflation from separable factors (WH_DEFL_FACTORED): the same solves
as with the dense vectors the factors represent, and against the oracle's DCG and the
direct solve; variable-c eigenvectors computed numerically and compressed by SVD."""
import numpy as np
import pytest

import workloads as wl
from oracle import discretization as disc, modes, krylov, wavesolve as ws, transfer as tr
from compress_modes import compress_modes
from _gpu import cuda, host, oracle_tp, relmx

pytestmark = pytest.mark.gpu


def _rotated_sine_set(n, omega, nd, seed=5):
    """The nd sine modes nearest resonance, each degenerate pair (a, b), (b, a) rotated by a
    random angle: still orthonormal eigenvectors, now of rank 2 on the grid."""
    sel, lam2 = modes.select_modes(2, n, omega, nd)
    sel = [tuple(int(v) for v in m) for m in sel]
    V = np.stack([modes.mode_nodal(2, n, m) for m in sel])
    rng = np.random.default_rng(seed)
    done = set()
    for i, m in enumerate(sel):
        j = sel.index((m[1], m[0])) if (m[1], m[0]) in sel else -1
        if j > i and i not in done:
            th = rng.uniform(0.2, 1.3)
            a, b = V[i].copy(), V[j].copy()
            V[i], V[j] = np.cos(th) * a + np.sin(th) * b, -np.sin(th) * a + np.cos(th) * b
            done |= {i, j}
    return V, np.asarray(lam2), len(done) // 2


@pytest.mark.parametrize("solver", ["dcg", "gmres", "bicgstab"])
def test_factored_matches_dense_and_oracle(solver):
    print(f"case factored {solver}", flush=True)
    import torch
    import paper_2606_31842_amd as wh
    n = 64
    e = modes.eig1d(n)
    omega = float(np.sqrt(e[6] + e[7]) * 1.0015)
    f = wl.gaussian(2, n, (0.41, 0.57), 0.08)
    V, lam2, npairs = _rotated_sine_set(n, omega, 10)
    assert npairs >= 2
    fx, fy, tm, ranks = compress_modes(V, tol=1e-12)
    assert max(ranks) == 2
    dfac = wh.factored_deflation(fx, fy, tm, lam2)
    dden = wh.Deflation(wh.WH_DEFL_DENSE_EXACT, V=torch.stack([cuda(v).reshape(-1) for v in V]), lambda2=lam2)
    kw = dict(solver=solver, tol=1e-10, max_iters=4000, restart=30)
    uf, inf_ = wh.solve(cuda(f), omega, defl=dfac, **kw)
    ud, ind = wh.solve(cuda(f), omega, defl=dden, **kw)
    print(f"factored iters {inf_['iters']} dense iters {ind['iters']} ranks {list(ranks)}", flush=True)
    assert inf_["status"] == 0 and ind["status"] == 0
    assert abs(inf_["iters"] - ind["iters"]) <= 1
    assert relmx(host(uf), host(ud)) < 1e-9
    U = disc.to_nodal(disc.direct_solve(disc.laplacian(2, n), omega, disc.to_interior(f)), 2, n)
    assert relmx(host(uf), U) < 1e-8
    if solver == "dcg":
        # the oracle's DCG with the dense W these factors represent
        L = disc.laplacian(2, n)
        tp = oracle_tp(2, n, omega)
        W = np.stack([disc.to_interior(v) for v in V], axis=1)
        b = ws.rhs(L, disc.to_interior(f), tp)
        _, oi = krylov.dcg(lambda v: ws.apply_A(L, v, tp), b, W, W * tr.mu_discrete(lam2, tp), tol=1e-10,
                           reproject=False)
        assert abs(inf_["iters"] - oi["iters"]) <= 2


def test_factored_variable_c_compressed_eigenvectors():
    """Variable c: eigenvectors of L_h from a shift-invert eigensolve near omega^2 (scipy,
    test data).  Kept to tau = 1e-10 the factored set reproduces DCG with the full vectors;
    compressed to tau = 1e-5 it reproduces the compression experiment of Section 4.3 (CG on
    the forcing deflated with the compressed vectors, stopping tolerance 1e-4): the same
    iteration count as with the full vectors."""
    print("case factored variable c", flush=True)
    import torch
    import paper_2606_31842_amd as wh
    from scipy.sparse.linalg import eigsh
    n = 64
    rng = np.random.default_rng(9)
    c2 = wl.config5_c2(n, rng)
    L = disc.laplacian(2, n, c2)
    omega = 19.3
    vals, vecs = eigsh(-L, k=12, sigma=omega ** 2, which="LM")
    lam2 = vals
    V = np.stack([disc.to_nodal(vecs[:, k], 2, n) for k in range(vecs.shape[1])])
    f = wl.gaussian(2, n, (0.37, 0.61), 0.07)
    U = disc.to_nodal(disc.direct_solve(L, omega, disc.to_interior(f)), 2, n)
    dden = wh.Deflation(wh.WH_DEFL_DENSE_EXACT, V=torch.stack([cuda(v).reshape(-1) for v in V]), lambda2=lam2)
    # full accuracy: DCG to 1e-9
    kw = dict(solver="dcg", tol=1e-9, max_iters=4000, c2=cuda(c2))
    ud, ind = wh.solve(cuda(f), omega, defl=dden, **kw)
    fx, fy, tm, ranks = compress_modes(V, tol=1e-10)
    uf, inf_ = wh.solve(cuda(f), omega, defl=wh.factored_deflation(fx, fy, tm, lam2), **kw)
    print(f"tau 1e-10: ranks {list(ranks)} iters {inf_['iters']} (dense {ind['iters']}) "
          f"err {relmx(host(uf), U):.1e}", flush=True)
    assert ind["status"] == 0 and inf_["status"] == 0
    assert abs(inf_["iters"] - ind["iters"]) <= 1
    assert relmx(host(ud), U) < 1e-6 and relmx(host(uf), U) < 1e-6
    assert max(ranks) < n - 1
    # the compression experiment: CG with f_d, tol 1e-4
    kw = dict(solver="cg", devd=1, tol=1e-4, max_iters=4000, c2=cuda(c2))
    ud, ind = wh.solve(cuda(f), omega, defl=dden, **kw)
    fx, fy, tm, ranks = compress_modes(V, tol=1e-5)
    uf, inf_ = wh.solve(cuda(f), omega, defl=wh.factored_deflation(fx, fy, tm, lam2), **kw)
    print(f"tau 1e-5, CG with f_d to 1e-4: ranks {list(ranks)} iters {inf_['iters']} (full {ind['iters']}) "
          f"err {relmx(host(uf), U):.1e} (full {relmx(host(ud), U):.1e})", flush=True)
    assert ind["status"] == 0 and inf_["status"] == 0
    assert inf_["iters"] == ind["iters"]
    assert max(ranks) <= 16


def test_factored_rejects_bad_input():
    import torch
    import paper_2606_31842_amd as wh
    n = 24
    sel, lam2 = modes.select_modes(2, n, 7.7, 2)
    V = np.stack([modes.mode_nodal(2, n, m) for m in sel])
    fx, fy, tm, _ = compress_modes(V, tol=1e-12)
    f = cuda(wl.gaussian(2, n, (0.4, 0.6), 0.1))
    bad = wh.factored_deflation(fx, fy, tm[::-1].copy(), lam2)          # decreasing term_mode
    with pytest.raises(wh.WaveHoltzError):
        wh.solve(f, 7.7, solver="dcg", defl=bad)
    gap = wh.factored_deflation(fx, fy, np.array([0, 0], dtype=np.int32), lam2)   # mode 1 missing
    with pytest.raises(wh.WaveHoltzError):
        wh.solve(f, 7.7, solver="dcg", defl=gap)


def test_factored_mixed_dcg():
    """Mixed precision with the factored set: the same iterate as with the dense columns
    (both step in FP32 and project in FP64), within the mixed-path bound of the direct solve."""
    import torch
    import paper_2606_31842_amd as wh
    n = 96
    e = modes.eig1d(n)
    omega = float(np.sqrt(e[9] + e[11]) * 1.001)
    f = wl.gaussian(2, n, (0.37, 0.6), 0.07)
    V, lam2, npairs = _rotated_sine_set(n, omega, 12)
    fx, fy, tm, ranks = compress_modes(V, tol=1e-12)
    dfac = wh.factored_deflation(fx, fy, tm, lam2)
    dden = wh.Deflation(wh.WH_DEFL_DENSE_EXACT, V=torch.stack([cuda(v).reshape(-1) for v in V]), lambda2=lam2)
    kw = dict(solver="dcg", tol=1e-9, max_iters=4000, precision="mixed")
    uf, inf_ = wh.solve(cuda(f), omega, defl=dfac, **kw)
    ud, ind = wh.solve(cuda(f), omega, defl=dden, **kw)
    U = disc.direct_solve_dst(2, n, omega, f)
    print(f"mixed factored iters {inf_['iters']} dense {ind['iters']} err {relmx(host(uf), U):.1e}", flush=True)
    assert inf_["status"] == 0 and ind["status"] == 0
    assert abs(inf_["iters"] - ind["iters"]) <= 2
    assert relmx(host(uf), U) < 2e-5 and relmx(host(uf), host(ud)) < 2e-5
