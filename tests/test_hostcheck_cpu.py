"""Host-side checks of libwaveholtz without a GPU (tests/hostcheck): the library's host code,
built without device code under AddressSanitizer and UBSan, drives every entry point
against a stand-in HIP runtime that checks every kernel launch (each kernel has a model) and
every copy against the buffers it touches (the index ranges each launch would reach are computed with
the kernels' own formulas).  The adjoint group replays the arguments of the GPU adjoint tests
(n = 24, checkpoints every 2, 5, 16 steps)."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HC = os.path.join(HERE, "hostcheck")

pytestmark = pytest.mark.skipif(not os.path.exists(os.path.join(HC, "build.py")), reason="hostcheck sources absent")


@pytest.fixture(scope="module")
def exe():
    import sys
    sys.path.insert(0, HC)
    import build as hcbuild
    return hcbuild.build()


@pytest.mark.parametrize("group", ["vjp", "solve", "filter", "batched"])
@pytest.mark.parametrize("seed", [1, 2])
def test_host_code_under_sanitizers(exe, group, seed):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, group, str(seed)], capture_output=True, text=True, env=env, timeout=600)
    tail = (r.stdout[-3000:] + "\n" + r.stderr[-6000:])
    assert r.returncode == 0, tail
    assert "HOSTCHECK OK" in r.stdout, tail
    # every kernel the library launches has a model: a launch no model checks is a failure
    assert "not modelled" not in r.stdout, tail
