"""Build the HIP library libpdfmc.so for gfx950 (in-tree, next to this file).

Flags:
  --offload-arch=gfx950         MI355X (CDNA4)
  -ffp-contract=off             no implicit fma: the FP64 kernels follow the
                                operation order of the step contract exactly
  -target-feature -packed-fp32-ops   no packed FP32 instructions
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpdfmc.so")
HIP_SOURCES = ["pdfmc_api.hip", "k_particle.hip", "k_scatter.hip", "k_nodes.hip", "k_sort.hip", "k_mg.hip", "k_direct.hip"]
CXX_SOURCES = ["pdfmc_mesh.cpp", "pdfmc_amg.cpp", "pdfmc_chol.cpp"]
ARCH = os.environ.get("PDFMC_ARCH", "gfx950")


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    obj_dir = os.path.join(os.path.dirname(HERE), "_build")
    os.makedirs(obj_dir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off"]
    dev = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    jobs = []
    for s in HIP_SOURCES:
        o = os.path.join(obj_dir, s.replace(".hip", ".o"))
        jobs.append([hipcc] + dev + common + ["-c", os.path.join(CSRC, s), "-o", o])
    for s in CXX_SOURCES:
        o = os.path.join(obj_dir, s.replace(".cpp", ".o"))
        jobs.append(["g++"] + common + ["-I/opt/rocm/include", "-c", os.path.join(CSRC, s), "-o", o])

    def run(cmd):
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        if verbose:
            print(r.stderr)
        return cmd[-1]

    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = list(ex.map(run, jobs))
    tmp = LIB + ".tmp"
    link = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(link)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
