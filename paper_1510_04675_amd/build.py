"""Build the HIP library libmsmc.so for gfx950 with hipcc (in-tree).

Every source under csrc/ is compiled to an object in parallel, then linked
into paper_1510_04675_amd/lib/libmsmc.so.  Device code is compiled with
packed fp32 instructions disabled; *_f32.hip units allow fused multiply-add
contraction and the others are compiled without it, except where a unit
enables it in its source (the fp64 HMC step and flow stage).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "lib")
LIB = os.path.join(OUT_DIR, "libmsmc.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["k_phase_f64.hip", "k_phase_f32.hip", "k_update.hip", "k_measure.hip", "k_hmc.hip", "k_hmc_f64.hip",
           "k_flow.hip", "k_flow_f64.hip", "k_prolong.hip", "capi.hip"]
ARCH = os.environ.get("MSMC_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", INCLUDE]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found; the MI355X library cannot be built")
    return p


def contract_flag(src: str) -> str:
    """fp32 translation units may fuse multiply-adds; all others are compiled
    without contraction so fp64 results follow the stated operation order."""
    return "-ffp-contract=fast" if src.endswith("_f32.hip") else "-ffp-contract=off"


def _compile(src: str, obj: str) -> None:
    cmd = [hipcc(), *FLAGS, contract_flag(src), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")


def build(jobs: int = 6) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    objdir = os.path.join(OUT_DIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in SOURCES]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda a: _compile(*a), zip(SOURCES, objs)))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("linking libmsmc.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
