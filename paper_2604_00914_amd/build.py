"""Compile the HIP library ``libafsi.so`` for gfx950 in-tree.

Every source under ``csrc/`` is compiled with hipcc into ``_build/`` (in parallel)
and linked into ``paper_2604_00914_amd/libafsi.so``.  Run ``python -m
paper_2604_00914_amd.build`` from the repository root.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libafsi.so")

ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]
# gfx950 device code: no packed FP32 instructions
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# per-source device flags: MFMA accumulators in ordinary VGPRs, so the k-loop carries
# them without copies to and from the accumulator registers
DEVICE_EXTRA = {"mfma_f64.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


# host-only sources (no HIP), built with the host compiler and OpenMP (libgomp):
# source -> [(object, extra flags)]; host_linalg.cpp twice, generic and AVX2/FMA
HOST_ONLY = {
    "host_linalg.cpp": [("host_linalg_generic.o", ["-DAFSI_ISA_NS=generic"]),
                        ("host_linalg_avx2.o", ["-DAFSI_ISA_NS=avx2", "-mavx2", "-mfma"])],
    "host_linalg_dispatch.cpp": [("host_linalg_dispatch.o", [])],
}
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fcx-limited-range", "-fopenmp",
              "-Wall"]


def _jobs():
    out = []
    for src in sources():
        for obj, extra in HOST_ONLY.get(src, [(os.path.splitext(src)[0] + ".o", None)]):
            out.append((src, obj, extra))
    return out


def _compile(job, verbose: bool):
    src, objname, extra = job
    obj = os.path.join(BUILD, objname)
    if extra is not None:
        cmd = [os.environ.get("CXX", "g++"), *HOST_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    else:
        cmd = [hipcc(), *COMMON, *DEVICE, *DEVICE_EXTRA.get(src, []), "-c", os.path.join(CSRC, src),
               "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{out}")
    if verbose and out.strip():
        print(out, file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda j: _compile(j, verbose), _jobs()))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-lgomp", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libafsi.so failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
