"""Build the host-only check program: libwaveholtz's sources compiled without device code
under AddressSanitizer + UBSan, linked with the stand-in HIP runtime (hip_stub.hip) and the
driver (driver.cpp).  Output: tests/hostcheck/_build/hostcheck.  CPU only."""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
from paper_2606_31842_amd import build as libbuild  # noqa: E402

OUT = os.path.join(HERE, "_build")
EXE = os.path.join(OUT, "hostcheck")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
# sanitizer flags apply to host code only
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]
COMMON = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-D_GLIBCXX_ASSERTIONS",
          "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    jobs = []
    srcs = [os.path.join(libbuild.CSRC, s) for s in libbuild.SOURCES] + [os.path.join(HERE, "hip_stub.hip")]
    for src in srcs:
        obj = os.path.join(OUT, os.path.splitext(os.path.basename(src))[0] + ".o")
        jobs.append([HIPCC, "--cuda-host-only", *COMMON, *SAN, "-c", src, "-o", obj])
    drv = os.path.join(OUT, "driver.o")
    jobs.append([CLANG, *COMMON, "-fsanitize=address,undefined", "-c", os.path.join(HERE, "driver.cpp"),
                 "-o", drv])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        return cmd, subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 4)) as ex:
        results = list(ex.map(run, jobs))
    bad = [(c, r) for c, r in results if r.returncode != 0]
    if bad:
        raise RuntimeError("\n".join(" ".join(c) + "\n" + r.stderr for c, r in bad))
    objs = [c[-1] for c, _ in results]
    # the host objects name the (absent) device code blobs; define empty ones
    undef = subprocess.run(["nm", "-u", *objs], capture_output=True, text=True, check=True).stdout
    blobs = sorted(set(re.findall(r"\b(__hip_fatbin_[0-9a-f]+)\b", undef)))
    stub_c = os.path.join(OUT, "fatbins.c")
    with open(stub_c, "w") as fh:
        for b in blobs:
            fh.write(f"char {b}[16];\n")
    fat_o = os.path.join(OUT, "fatbins.o")
    subprocess.run(["/opt/rocm/llvm/bin/clang", "-c", stub_c, "-o", fat_o], check=True)
    link = [CLANG, "-fsanitize=address,undefined", *objs, fat_o, "-o", EXE]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(" ".join(link) + "\n" + r.stderr)
    return EXE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
