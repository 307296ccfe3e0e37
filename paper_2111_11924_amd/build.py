"""Build the HIP library libpmk.so (gfx950) in-tree with hipcc.

    python -m paper_2111_11924_amd.build [--jobs N] [--incremental]

Each source is compiled to an object in _build/obj, then linked into
paper_2111_11924_amd/libpmk.so.  Device code is built for gfx950 only.
--incremental recompiles only objects older than their source or than any
header of csrc/ and include/ (every header is taken as a dependency of every
source); the default rebuilds everything.

Code alignment: after compiling, the build reads where each kernel's
v_mad_u64_u32 instructions landed (llvm-objdump of the objects' own gfx950
code) and recompiles a source whose kernels have more than 60 % of them at addresses
4 modulo 8, with those kernels listed in PMK_CODE_PAD (kernels_impl.hpp: they
then start with one 4-byte s_nop).  The decisions are kept in
csrc/code_pad.json, which every build starts from: with unchanged sources and
compiler no kernel needs a second compile.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import subprocess
import sys
import tempfile
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


LLVM = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin")
# the padding decisions, kept beside the sources so that a build starts from
# them: {"pad": {source: [code_id, ...]}, "fixed": {source: [code_id, ...]}}
# ("fixed": kernels the 4 bytes do not move)
PADS = os.path.join(CSRC, "code_pad.json")
# kernel kinds: the numbers of CodeKind in kernels_impl.hpp
CODE_KIND = {"encrypt_kernel": 1, "halves_kernel": 2, "halves_joint_kernel": 3, "halves_lanes_kernel": 4,
             "halves_lanes_joint_kernel": 5, "garner_kernel": 6, "garner_lds_kernel": 7, "batch_wide_kernel": 8,
             "mp_part_kernel": 9, "mp_garner_kernel": 10, "miller_rabin_kernel": 11}


def _headers_mtime() -> float:
    paths = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".inc", ".h"))]
    inc = os.path.join(ROOT, "include")
    paths += [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]
    return max(os.path.getmtime(p) for p in paths)


def _compile(src: str, incremental: bool = False, hdr_mtime: float = 0.0, pads=()) -> str:
    path = os.path.join(CSRC, src)
    out = os.path.join(OBJ, src + ".o")
    if incremental and os.path.exists(out):
        if os.path.getmtime(out) > max(os.path.getmtime(path), hdr_mtime):
            return out
    tmp = out + f".{os.getpid()}.tmp"
    pad = [f"-DPMK_CODE_PAD={','.join(f'{i}u' for i in sorted(pads))}"] if pads else []
    cmd = [HIPCC] + COMMON + pad + DEVICE + ["-x", "hip", "-c", path, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def _code_id(symbol: str):
    """code_id of a kernel from its mangled name (pmk::<kind><args...>), or None."""
    m = re.match(r"_ZN3pmk(\d+)", symbol)
    if not m:
        return None
    n = int(m.group(1))
    name = symbol[m.end():m.end() + n]
    if name not in CODE_KIND:
        return None
    t = re.match(r"I((?:Li-?\d+E)+)E", symbol[m.end() + n:])  # template arguments <int, ...>
    args = [int(a) for a in re.findall(r"Li(-?\d+)E", t.group(1))] if t else []
    a, b = (args + [0, 0])[:2]
    return CODE_KIND[name] * 1000000 + a * 10 + b


def mad_alignment(obj: str) -> dict:
    """{code_id: (multiply-adds, of them at 4 modulo 8)} over the kernels of an object."""
    with tempfile.TemporaryDirectory() as tmp:
        fb, co = os.path.join(tmp, "fb.bin"), os.path.join(tmp, "dev.co")
        subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", f".hip_fatbin={fb}", obj, os.devnull],
                       check=True, capture_output=True)
        subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--type=o",
                        f"--targets=hipv4-amdgcn-amd-amdhsa--{ARCH}", f"--input={fb}", f"--output={co}", "--unbundle"],
                       check=True, capture_output=True)
        text = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", f"--mcpu={ARCH}", co],
                              check=True, capture_output=True, text=True).stdout
    res, cur = {}, None
    for line in text.splitlines():
        m = re.match(r"^[0-9a-f]+ <(.*)>:$", line)
        if m:
            cur = _code_id(m.group(1))
            if cur is not None:
                res.setdefault(cur, [0, 0])
            continue
        if cur is None or "v_mad_u64_u32" not in line:
            continue
        a = re.search(r"//\s*([0-9A-F]+):", line)
        if a:
            res[cur][0] += 1
            res[cur][1] += int(a.group(1), 16) % 8 != 0
    return res


def _align_tools() -> bool:
    return all(os.path.exists(os.path.join(LLVM, t)) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-objdump"))


def build_probe() -> str:
    tmp = PROBE + f".{os.getpid()}.tmp"
    subprocess.check_call([HIPCC, "-O3", "-std=c++17"] + DEVICE + [os.path.join(CSRC, "mad_rate.hip"), "-o", tmp])
    os.replace(tmp, PROBE)
    return PROBE


def build(jobs: int = 8, verbose: bool = True, incremental: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    hdr = _headers_mtime()
    pads, fixed = {}, {}
    if os.path.exists(PADS):
        with open(PADS) as f:
            saved = json.load(f)
        pads = {k: set(v) for k, v in saved.get("pad", {}).items()}
        fixed = {k: set(v) for k, v in saved.get("fixed", {}).items()}
    first = {k: set(v) for k, v in pads.items()}, {k: set(v) for k, v in fixed.items()}
    kernels = [s for s in SOURCES if s.endswith(".hip")]
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        probe = None
        if not (incremental and os.path.exists(PROBE)
                and os.path.getmtime(PROBE) > os.path.getmtime(os.path.join(CSRC, "mad_rate.hip"))):
            probe = ex.submit(build_probe)
        objs = list(ex.map(lambda s: _compile(s, incremental, hdr, pads.get(s, ())), SOURCES))
        if _align_tools():
            # kernels with most of their multiply-adds at 4 modulo 8 change padding
            scan = lambda s: mad_alignment(os.path.join(OBJ, s + ".o"))
            before = dict(zip(kernels, ex.map(scan, kernels)))
            # more than 60 %: a kernel nearer half and half (its code keeps no one
            # parity) is left as it is; moving such a kernel measured either way
            # (the 2048-bit encryption, 54 % -> 46 %, took 16 % longer per
            # launch in the 1 MiB workload)
            flips = {s: {i for i, (n, odd) in before[s].items()
                         if n >= 64 and 5 * odd > 3 * n and i not in fixed.get(s, ())} for s in kernels}
            flips = {s: f for s, f in flips.items() if f}
            for s, f in flips.items():
                pads[s] = pads.get(s, set()) ^ f
            list(ex.map(lambda s: _compile(s, False, hdr, pads.get(s, ())), flips))
            after = dict(zip(flips, ex.map(scan, flips)))
            # a kernel whose multiply-adds the 4 bytes did not move (a loop
            # aligned on its own) goes back to its first form
            back = {s: {i for i in f if after[s].get(i, [0, 0])[1] >= before[s][i][1]} for s, f in flips.items()}
            back = {s: b for s, b in back.items() if b}
            for s, b in back.items():
                pads[s] ^= b
                fixed[s] = fixed.get(s, set()) | b
            list(ex.map(lambda s: _compile(s, False, hdr, pads.get(s, ())), back))
            if verbose:
                for s in flips:
                    res = scan(s) if s in back else after[s]
                    print(f"code alignment: {s}: {len(pads.get(s, ()))} kernel(s) padded, "
                          f"{sum(v[1] for v in res.values())} of {sum(v[0] for v in res.values())} "
                          f"multiply-adds at 4 modulo 8")
            if (pads, fixed) != first:
                with open(PADS, "w") as f:
                    json.dump({"pad": {k: sorted(v) for k, v in sorted(pads.items()) if v},
                               "fixed": {k: sorted(v) for k, v in sorted(fixed.items()) if v}}, f, indent=1)
                    f.write("\n")
        elif verbose:
            print("code alignment: llvm tools not found, kernels left unpadded")
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
