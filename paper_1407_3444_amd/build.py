"""Build libchi0.so for gfx950 with hipcc (in-tree, next to this file).

Every source is compiled to its own object in parallel (each object carries its own device code),
then the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libchi0.so")
OBJDIR = os.path.join(os.path.dirname(HERE), "_build", "libchi0")
SOURCES = ["k_tetra_dyn.hip", "k_tetra_list.hip", "k_tetra_batch.hip", "k_tetra_misc.hip", "k_contract.hip",
           "k_reduce.hip", "k_kk.hip", "k_check.hip", "chi0_api.cpp", "chi0_batch.cpp", "chi0_iw.cpp",
           "chi0_noalloc.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # no packed-FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def _run(cmd):
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    noise = "unknown target feature"
    out = "\n".join(l for l in res.stdout.splitlines() if noise not in l and "packed-fp32-ops" not in l)
    return res.returncode, out


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    tag = ".%d" % os.getpid()
    jobs = []
    for s in SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(s)[0] + tag + ".o")
        jobs.append(([hipcc()] + HIPCC_FLAGS + ["-c", os.path.join(CSRC, s), "-o", obj], obj))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "0") or 0) or (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(lambda j: _run(j[0]), jobs))
    objs = [o for _, o in jobs]
    try:
        for (cmd, _), (rc, out) in zip(jobs, results):
            if verbose:
                print(" ".join(cmd), flush=True)
            if rc != 0:
                raise RuntimeError("hipcc failed:\n" + out)
            if verbose and out.strip():
                print(out)
        tmp = LIB + ".tmp%d" % os.getpid()
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        rc, out = _run(link)
        if rc != 0:
            raise RuntimeError("hipcc link failed:\n" + out)
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
