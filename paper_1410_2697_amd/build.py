"""Build the HIP library ``libmfh.so`` in-tree for gfx950.

Usage: python -m paper_1410_2697_amd.build   (or build() from Python).
Each source is compiled to an object under ``_build/`` (in parallel), then
linked; every call compiles every source again.
"""
from __future__ import annotations

import json
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmfh.so")
OBJ = os.path.join(os.path.dirname(HERE), "_build")
SOURCES = ["hostpool.cpp", "symbolic.cpp", "prof.cpp", "server.cpp", "api.cpp", "kernels.hip", "numeric.hip",
           "testing.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions are kept out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    return r.returncode, err


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = []
    for s in srcs:
        o = os.path.join(OBJ, s + ".o")
        extra = ["-Rpass-analysis=kernel-resource-usage"] if s.endswith(".hip") else []
        jobs.append((o, [cc] + FLAGS + extra + ["-c", "-o", o, os.path.join(CSRC, s)]))
    if verbose:
        for _, c in jobs:
            print(" ".join(c), flush=True)
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(workers) as ex:
        res = list(ex.map(lambda j: _run(j[1]), jobs))
    errs = [e for (rc, e) in res if rc != 0]
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    _write_resources([e for (_, e) in res])
    link = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + [o for o, _ in jobs]
    rc, err = _run(link)
    if rc != 0:
        raise RuntimeError("link failed:\n" + err)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _write_resources(logs):
    """Per-kernel registers, scratch and occupancy from the compiler's
    resource remarks, to ``_build/kernel_resources.json`` (a kernel that
    spills its register-resident rows to scratch memory runs many times
    slower, and the host tests check that none does)."""
    out, name = {}, None
    for log in logs:
        for line in log.splitlines():
            m = re.search(r"remark: Function Name: (\S+)", line)
            if m:
                name = m.group(1)
                out[name] = {}
                continue
            m = re.search(r"remark:\s+(VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)", line)
            if m and name:
                out[name][m.group(1).split(" ")[0]] = int(m.group(2))
    with open(os.path.join(OBJ, "kernel_resources.json"), "w") as f:
        json.dump(out, f, indent=0, sort_keys=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
