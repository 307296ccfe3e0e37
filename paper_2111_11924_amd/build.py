"""Build the HIP library libpmk.so (gfx950) in-tree with hipcc.

    python -m paper_2111_11924_amd.build [--jobs N] [--incremental]

Each source is compiled to an object in _build/obj, then linked into
paper_2111_11924_amd/libpmk.so.  Device code is built for gfx950 only.
--incremental recompiles only objects older than their source or than any
header of csrc/ and include/ (every header is taken as a dependency of every
source); the default rebuilds everything.
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
           "kprime.hip", "kmp.hip", "kjoint.hip", "klanes.hip", "kjlanes.hip", "noalloc.hip", "dispatch.cpp", "pmk_api.cpp", "mp_api.cpp", "keyprep.cpp", "server.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-mllvm", "-pragma-unroll-threshold=400000", "-fPIC", "-Wall", "-Wno-unused-result", f"-I{os.path.join(ROOT, 'include')}"]
# device code: gfx950 only; packed-FP32 instruction selection off
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _headers_mtime() -> float:
    paths = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".inc", ".h"))]
    inc = os.path.join(ROOT, "include")
    paths += [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]
    return max(os.path.getmtime(p) for p in paths)


def _compile(src: str, incremental: bool = False, hdr_mtime: float = 0.0) -> str:
    path = os.path.join(CSRC, src)
    out = os.path.join(OBJ, src + ".o")
    if incremental and os.path.exists(out):
        if os.path.getmtime(out) > max(os.path.getmtime(path), hdr_mtime):
            return out
    tmp = out + f".{os.getpid()}.tmp"
    cmd = [HIPCC] + COMMON + DEVICE + ["-x", "hip", "-c", path, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build_probe() -> str:
    tmp = PROBE + f".{os.getpid()}.tmp"
    subprocess.check_call([HIPCC, "-O3", "-std=c++17"] + DEVICE + [os.path.join(CSRC, "mad_rate.hip"), "-o", tmp])
    os.replace(tmp, PROBE)
    return PROBE


def build(jobs: int = 8, verbose: bool = True, incremental: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    hdr = _headers_mtime()
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        probe = None
        if not (incremental and os.path.exists(PROBE)
                and os.path.getmtime(PROBE) > os.path.getmtime(os.path.join(CSRC, "mad_rate.hip"))):
            probe = ex.submit(build_probe)
        objs = list(ex.map(lambda s: _compile(s, incremental, hdr), SOURCES))
        if probe is not None:
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
    ap.add_argument("--incremental", action="store_true")
    a = ap.parse_args()
    build(a.jobs, incremental=a.incremental)
    sys.exit(0)
