"""Builds libskolem.so (host C++ + gfx950 kernels) in-tree with hipcc.

    python -m paper_1507_00315_amd.build        # or build() from Python

Every HIP source is compiled for gfx950 only, with packed-FP32 instructions
disabled and FP contraction off (the exact fp64 residue arithmetic relies on
each rounding written in the source).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libskolem.so")
# The issue-rate calibration program (not part of the library): the cost
# model of the tempering kernel, run by `bench.py --issue-calibration`.
PROBE = os.path.join(HERE, "issue_probe")

SOURCES = ["host.cpp", "pt_host.cpp", "mlp_host.cpp", "exact_v1.hip", "pt.hip", "mlp.hip"]

# Persistent batched kernels: (group, primes per work item) per translation
# unit; group 1 (the mixed-instance workload) also with one prime per work
# item, an axis of the autotuner.
BATCH_UNITS = [(0, 0), (1, 0), (1, 1), (2, 0), (3, 0)]

# Tuned kernel specialisations: (variant, n_min, n_max) per translation unit,
# so they compile in parallel.
V2_UNITS = [(v, lo, hi) for v in (0, 1, 2) for lo, hi in ((12, 15), (16, 18), (19, 21), (22, 24),
                                                           (25, 27), (28, 30), (31, 32))]
# The inclusion-exclusion sum (Sec. 2, third approach), tuned body: n = 12..22.
LARSEN_UNITS = [(v, lo, hi) for v in (0, 1, 2) for lo, hi in ((12, 16), (17, 19), (20, 22))]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compiles every source to an object (in parallel) and links the library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    units = [(src, src + ".o", []) for src in SOURCES]
    for v, lo, hi in V2_UNITS:
        units.append(("exact_v2_inst.hip", f"exact_v2_{v}_{lo}_{hi}.o",
                      [f"-DSK_V2_VARIANT={v}", f"-DSK_V2_NMIN={lo}", f"-DSK_V2_NMAX={hi}"]))
    for g, ppi in BATCH_UNITS:
        units.append(("exact_batch.hip", f"exact_batch_{g}_{ppi}.o", [f"-DSK_BATCH_GROUP={g}", f"-DSK_BATCH_PPI={ppi}"]))
    for v, lo, hi in LARSEN_UNITS:
        units.append(("exact_v2_inst.hip", f"larsen_v2_{v}_{lo}_{hi}.o",
                      [f"-DSK_V2_VARIANT={v}", f"-DSK_V2_NMIN={lo}", f"-DSK_V2_NMAX={hi}", "-DSK_V2_LARSEN=1"]))
    for src, oname, defs in units:
        obj = os.path.join(objdir, oname)
        objs.append(obj)
        cmd = [hipcc()] + HIPCC_FLAGS + defs + ["-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src),
                                                "-o", obj]
        if src.endswith(".cpp"):
            cmd = cmd[:1] + ["-x", "hip"] + cmd[1:]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((oname, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while sum(1 for _, p in procs if p.poll() is None) >= jobs:
            time.sleep(0.2)
    probe_cmd = [hipcc()] + HIPCC_FLAGS + ["-o", PROBE + ".tmp", os.path.join(CSRC, "issue_probe.hip")]
    if verbose:
        print(" ".join(probe_cmd), flush=True)
    procs.append(("issue_probe.hip", subprocess.Popen(probe_cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    errors = []
    for src, p in procs:
        out, _ = p.communicate()
        text = "\n".join(ln for ln in out.decode(errors="replace").splitlines()
                         if "packed-fp32-ops" not in ln and ln.strip())
        if p.returncode != 0:
            errors.append(f"--- {src}\n{text}")
        elif verbose and text.strip():
            print(text)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    os.replace(PROBE + ".tmp", PROBE)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
