"""Builds the HIP library libmhr.so for gfx950 in-tree (hipcc, no JIT cache).

Every HIP source is compiled with packed-FP32 instruction generation
disabled (-Xclang -target-feature -Xclang -packed-fp32-ops).

``--phase-clocks`` builds the profiling variant libmhr_phase.so instead:
the same sources with MHR_PHASE_CLOCKS defined, so that the gather kernel
records per-phase wall-clock ticks (mhr_debug_phase_ticks).  The binding
loads it when MHR_LIBRARY names it."""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmhr.so")
PHASE_LIB = os.path.join(HERE, "libmhr_phase.so")
SOURCES = ["mhr_api.hip", "mhr_graph.hip", "mhr_query.hip", "mhr_plan.hip", "mhr_pruner.hip", "mhr_scan.hip", "mhr_files.hip", "mhr_beam.hip", "mhr_wide.hip"]
ARCH = os.environ.get("MHR_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I", INCLUDE, "-I", CSRC]


def build(verbose: bool = False, phase_clocks: bool = False) -> str:
    out_lib = PHASE_LIB if phase_clocks else LIB
    defines = ["-DMHR_PHASE_CLOCKS"] if phase_clocks else []
    objdir = os.path.join(HERE, "_build_phase" if phase_clocks else "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = ["hipcc", *HIPCC_FLAGS, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(text)
        elif verbose and text.strip():
            sys.stderr.write(text)
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    tmp = out_lib + ".tmp"
    subprocess.check_call(["hipcc", f"--offload-arch={ARCH}", "-shared", "-o", tmp, *objs])
    os.replace(tmp, out_lib)
    return out_lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, phase_clocks="--phase-clocks" in sys.argv))
