"""Build libxf.so for gfx950 with hipcc (in-tree, no JIT).

    python -m paper_2403_05910_amd.build            # build
    python -m paper_2403_05910_amd.build --report   # also print kernel resource usage

Two objects per species count (xf_ns.hip and xf_react.hip with -DXF_NS=N) so the heavy
template instantiations compile in parallel.
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libxf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
MAX_NS = 9

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # no packed-FP32 instructions (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(PKG, "..", "include"),
]


def _units():
    units = [("xf_api.hip", "xf_api.o", []), ("xf_misc.hip", "xf_misc.o", [])]
    for n in range(1, MAX_NS + 1):
        units.append(("xf_ns.hip", f"xf_ns{n}.o", [f"-DXF_NS={n}"]))
        # the reaction kernel without machine loop-invariant code motion (the
        # reason is at the top of xf_react.hip)
        units.append(("xf_react.hip", f"xf_react{n}.o", [f"-DXF_NS={n}", "-mllvm", "-disable-machine-licm"]))
    return units


def _compile(unit, report):
    src, obj, extra = unit
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, obj)]
    if report:
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    p = subprocess.run(cmd, capture_output=True, text=True)
    return unit, p.returncode, p.stdout + p.stderr


def build(report=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda u: _compile(u, report), _units()))
    failed = [(u, out) for (u, rc, out) in results if rc != 0]
    for (u, rc, out) in results:
        if report or rc != 0:
            lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l]
            if lines:
                sys.stderr.write(f"--- {u[1]}\n" + "\n".join(lines) + "\n")
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(u[1] for u, _ in failed))
    objs = [os.path.join(BUILD, u[1]) for u in _units()]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--report", action="store_true")
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args()
    print(build(report=a.report, jobs=a.j))
