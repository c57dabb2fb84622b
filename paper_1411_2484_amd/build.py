"""Build the gfx950 HIP library libphprng.so in-tree with hipcc.

Usage: python -m paper_1411_2484_amd.build  (or call build()).

The instruction-rate probe behind the measured per-class VALU rates is a
measurement tool, not part of the library: build it on its own with
python -m paper_1411_2484_amd.build --probe  (writes paper_1411_2484_amd/probe_rates).
"""

from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libphprng.so")
SOURCES = ["kernels.hip", "runtime.cpp", "hostmath.cpp", "server.cpp", "battery.hip", "battery.cpp", "pattern.hip", "phist.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def _run(cmd, what, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on " + what)


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compiles every source (in parallel, `jobs` at a time; 0: up to 8) and
    links libphprng.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    cmds = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmds.append(([hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *lang, "-c",
                      os.path.join(CSRC, src), "-o", obj], src))
        objs.append(obj)
    workers = jobs if jobs > 0 else max(1, min(8, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as pool:
        for f in [pool.submit(_run, cmd, what, verbose) for cmd, what in cmds]:
            f.result()
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


def build_probe(verbose: bool = False) -> str:
    """Builds the standalone instruction-rate probe (csrc/probe_rates.hip)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    probe = os.path.join(HERE, "probe_rates")
    _run([hipcc, *HIPCC_FLAGS, "-o", probe + ".tmp", os.path.join(CSRC, "probe_rates.hip")], "probe_rates.hip",
         verbose)
    os.replace(probe + ".tmp", probe)
    return probe


if __name__ == "__main__":
    print(build_probe(verbose=True) if "--probe" in sys.argv[1:] else build(verbose=True))
