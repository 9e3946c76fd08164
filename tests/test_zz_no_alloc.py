"""GPU check of wh_apply_filter_noalloc (the filter without a workspace argument, running in
the library's fixed device scratch) against wh_apply_filter with a caller workspace, called
through the C ABI: two calls in a row, the second on a smaller grid, in both precisions, with
and without variable c and forcing; one case also against the oracle's filter."""
import numpy as np
import pytest

import workloads as wl
from oracle import discretization as disc, timeparams as tpm, wavesolve as ws
from _gpu import cuda, host

pytestmark = pytest.mark.gpu


def _inputs(n, varc, seed):
    v = wl.random_nodal(2, n, seed)
    f = wl.gaussian(2, n, (0.4, 0.55), 0.1)
    c2 = None
    if varc:
        rng = np.random.default_rng(seed)
        c = 1.0 + wl.gaussian_sum_field(2, n, rng.uniform(-0.2, 0.2, 3), rng.uniform(0.3, 0.7, (3, 2)), 0.15)
        c2 = c * c
    return v, f, c2


@pytest.mark.parametrize("precision", ["f64", "mixed"])
@pytest.mark.parametrize("varc", [False, True])
@pytest.mark.parametrize("forcing", [False, True])
def test_noalloc_matches_workspace_filter_twice(precision, varc, forcing):
    import paper_2606_31842_amd as wh
    for n, omega, k, shape in [(150, 31.7, 8, 1), (61, 13.2, 6, 2)]:   # second call: smaller grid
        print(f"noalloc case {precision} varc={varc} forcing={forcing} n={n}", flush=True)
        v, f, c2 = _inputs(n, varc, seed=n)
        cmax = 1.0 if c2 is None else float(np.sqrt(c2.max()))
        kw = dict(precision=precision, k_fuse=k, k_shape=shape, c_max=cmax)
        vd, fd = cuda(v), (cuda(f) if forcing else None)
        cd = None if c2 is None else cuda(c2)
        ref, _ = wh.apply_filter(vd, omega, f=fd, c2=cd, **kw)
        got, info = wh.apply_filter_noalloc(vd, omega, f=fd, c2=cd, **kw)
        r, g = host(ref), host(got)
        assert info["k_fuse"] == k
        diff = np.abs(g - r).max() / np.abs(r).max()
        print(f"  max rel diff {diff:.2e} bit-identical {np.array_equal(g, r)}", flush=True)
        assert diff <= 1e-13


def test_noalloc_autotuned_choice_and_oracle():
    # without k_fuse the call takes the autotuner's cached choice from the workspace call
    import paper_2606_31842_amd as wh
    n, omega = 96, 21.4
    v, f, c2 = _inputs(n, True, seed=3)
    cmax = float(np.sqrt(c2.max()))
    ref, iref = wh.apply_filter(cuda(v), omega, f=cuda(f), c2=cuda(c2), c_max=cmax)
    got, igot = wh.apply_filter_noalloc(cuda(v), omega, f=cuda(f), c2=cuda(c2), c_max=cmax)
    assert (igot["k_fuse"], igot["k_rows"], igot["k_waves"]) == (iref["k_fuse"], iref["k_rows"], iref["k_waves"])
    assert np.abs(host(got) - host(ref)).max() <= 1e-13 * np.abs(host(ref)).max()
    L = disc.laplacian(2, n, c2)
    tp = tpm.time_parameters(omega, 1.0 / n, cmax)
    want = ws.wave_filter(L, disc.to_interior(v), disc.to_interior(f), tp)
    err = np.linalg.norm(disc.to_interior(host(got)) - want) / np.linalg.norm(want)
    print(f"noalloc vs oracle {err:.2e}", flush=True)
    assert err < 1e-12


def test_noalloc_rejects_grids_beyond_its_scratch():
    import paper_2606_31842_amd as wh
    v = cuda(np.zeros((1101, 1101)))
    with pytest.raises(wh.WaveHoltzError) as e:
        wh.apply_filter_noalloc(v, 50.0, precision="mixed")
    assert e.value.status == wh._native.WH_EWORKSPACE


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_noalloc_fourth_order_matches_workspace_filter_twice(precision):
    # fourth order (c = 1) runs the blocked radius-2 launches in the same fixed scratch
    import paper_2606_31842_amd as wh
    for n, omega, k in [(150, 31.7, 4), (61, 13.2, 2)]:
        print(f"noalloc order-4 case {precision} n={n} K={k}", flush=True)
        v, f, _ = _inputs(n, False, seed=n + 1)
        vd, fd = cuda(v), cuda(f)
        ref, iref = wh.apply_filter(vd, omega, f=fd, precision=precision, k_fuse=k, order=4)
        got, info = wh.apply_filter_noalloc(vd, omega, f=fd, precision=precision, k_fuse=k, order=4)
        assert info["k_fuse"] == iref["k_fuse"] == k
        r, g = host(ref), host(got)
        diff = np.abs(g - r).max() / np.abs(r).max()
        print(f"  max rel diff {diff:.2e} bit-identical {np.array_equal(g, r)}", flush=True)
        assert diff <= 1e-13
