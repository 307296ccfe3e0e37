"""Build the HIP library libpmk.so (gfx950) in-tree with hipcc.

    python -m paper_2111_11924_amd.build [--jobs N]

Each source is compiled to an object in _build/obj, then linked into
paper_2111_11924_amd/libpmk.so.  Device code is built for gfx950 only.
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(PKG, "libpmk.so")
PROBE = os.path.join(ROOT, "_build", "mad_rate")  # VALU issue-rate probe (python -m paper_2111_11924_amd.peak)

SOURCES = ["k8192.hip", "k6144.hip", "kbatch.hip", "k4096.hip", "k3072.hip", "k2048.hip", "k1024.hip", "k512.hip", "k256.hip", "k128.hip",
           "kprime.hip", "kmp.hip", "kjoint.hip", "dispatch.cpp", "pmk_api.cpp", "mp_api.cpp", "keyprep.cpp", "server.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-mllvm", "-pragma-unroll-threshold=400000", "-fPIC", "-Wall", "-Wno-unused-result", f"-I{os.path.join(ROOT, 'include')}"]
# device code: gfx950 only; packed-FP32 instruction selection off
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    out = os.path.join(OBJ, src + ".o")
    cmd = [HIPCC] + COMMON + DEVICE + ["-x", "hip", "-c", path, "-o", out]
    subprocess.check_call(cmd)
    return out


def build_probe() -> str:
    tmp = PROBE + f".{os.getpid()}.tmp"
    subprocess.check_call([HIPCC, "-O3", "-std=c++17"] + DEVICE + [os.path.join(CSRC, "mad_rate.hip"), "-o", tmp])
    os.replace(tmp, PROBE)
    return PROBE


def build(jobs: int = 8, verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        probe = ex.submit(build_probe)
        objs = list(ex.map(_compile, SOURCES))
        probe.result()
    tmp = LIB + f".{os.getpid()}.tmp"
    subprocess.check_call([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    a = ap.parse_args()
    build(a.jobs)
    sys.exit(0)
