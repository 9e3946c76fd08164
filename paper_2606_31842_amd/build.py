"""Build libwaveholtz.so for gfx950 with hipcc (in-tree, next to this file).

Each source is compiled to an object in parallel (build folder ``_build`` beside this
file), then the objects are linked into the shared library."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwaveholtz.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["wh_stencil.hip", "wh_fused.hip", "wh_fused_first.hip", "wh_fused_last.hip", "wh_fused3d.hip",
           "wh_blas.hip", "wh_batched.hip", "wh_march4.hip", "wh_adjoint.hip", "wh_api.hip"]

CFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]
LDFLAGS = ["--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,--no-undefined"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(HERE, "..", "include")]
    jobs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        if not os.path.exists(src):
            raise FileNotFoundError(src)
        jobs.append((src, os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o")))

    def compile_one(job):
        src, obj = job
        cmd = [hipcc, *CFLAGS, *inc, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        return src, r

    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(compile_one, jobs))
    failed = [(src, r) for src, r in results if r.returncode != 0]
    for src, r in results:
        msg = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
        if msg.strip() and (verbose or r.returncode != 0):
            print(msg, file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(os.path.basename(s) for s, _ in failed))
    tmp = LIB + ".tmp"
    cmd = [hipcc, *LDFLAGS, *[o for _, o in jobs], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
