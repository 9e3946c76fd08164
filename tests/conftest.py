import faulthandler
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_fault_file = None
_config = None


def pytest_configure(config):
    global _config
    _config = config
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.hookimpl(trylast=True)
def pytest_sessionstart(session):
    # A native abort inside a GPU test (the HIP runtime's message on a device fault, a C++
    # terminate) should be the last thing in the log.  pytest's own fault handler dumps every
    # thread's stack and the list of loaded modules to stderr after it, which pushes the
    # message out of a log tail; send that dump to a file instead.
    global _fault_file
    path = os.environ.get("WH_FAULT_LOG", os.path.join(ROOT, "gpurun_out", "pytest_faulthandler.log"))
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        _fault_file = open(path, "w")
        faulthandler.enable(file=_fault_file, all_threads=True)
    except OSError:
        _fault_file = None


def pytest_runtest_logstart(nodeid, location):
    # name each test before it runs, so that a crash inside it is attributable from the log
    tr = _config.pluginmanager.getplugin("terminalreporter") if _config is not None else None
    if tr is not None:
        tr.write_line(f"[start] {nodeid}", flush=True)


@pytest.hookimpl(wrapper=True, trylast=True)
def pytest_runtest_call(item):
    # GPU tests run with output capture off: what they and the native runtime print goes
    # straight to the log (a captured message is lost if the process aborts)
    if item.get_closest_marker("gpu") is None:
        return (yield)
    capman = item.config.pluginmanager.getplugin("capturemanager")
    if capman is None:
        return (yield)
    with capman.global_and_fixture_disabled():
        return (yield)
