"""Compile the HIP library in-tree: ``python -m paper_2606_07099_amd.build``.

Produces ``paper_2606_07099_amd/libsablepf.so`` for gfx950 with hipcc.  Packed
FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsablepf.so")
SOURCES = ["pf_kernels.hip", "pf_operators.hip", "pf_operator_static.hip", "pf_api.cpp", "symbolic.cpp",
           "operators.cpp"]
ARCH = os.environ.get("SABLE_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


LIB_PHASES = os.path.join(HERE, "libsablepf_phases.so")
OBJ_DIR = os.path.join(HERE, "_build")


def _flags():
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))


def build(verbose: bool = False) -> str:
    """Compiles every source (in parallel) and links two libraries: the
    production one and the measurement variant whose Newton kernel carries
    per-phase wall-clock counters (-DSABLE_PHASE_CLOCKS)."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJ_DIR, exist_ok=True)
    jobs = [(src, os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o"), []) for src in SOURCES]
    jobs.append(("pf_kernels.hip", os.path.join(OBJ_DIR, "pf_kernels_phases.o"), ["-DSABLE_PHASE_CLOCKS"]))
    cmds = [[hipcc(), *_flags(), *extra, "-c", os.path.join(CSRC, src), "-o", obj] for src, obj, extra in jobs]
    workers = max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    objs = [obj for _, obj, extra in jobs if not extra]
    phase_objs = [o if not o.endswith(os.sep + "pf_kernels.o") else jobs[-1][1] for o in objs]
    for out, ob in ((LIB, objs), (LIB_PHASES, phase_objs)):
        tmp = out + ".tmp"
        _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *ob, "-o", tmp], verbose)
        os.replace(tmp, out)
    build_abi_check(verbose)
    return LIB


ABI_CHECK = os.path.join(HERE, "abi_check")


def build_abi_check(verbose: bool = False) -> str:
    """The plain C client of the ABI (``csrc/abi_check.c``), linked against the
    library next to it; the tests run it as a child process."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler found")
    tmp = ABI_CHECK + ".tmp"
    cmd = [cc, "-std=c11", "-O2", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
           "-I", os.path.join(ROOT, "include"), os.path.join(CSRC, "abi_check.c"), "-o", tmp,
           "-L", HERE, "-lsablepf", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(rocm, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("C client build failed")
    os.replace(tmp, ABI_CHECK)
    return ABI_CHECK


if __name__ == "__main__":
    print(build(verbose=True))
