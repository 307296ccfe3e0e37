#!/usr/bin/env python3
"""Benchmark of the PMKRSA hot path on one MI355X.

Workload (one "step"): RSA encryption and CRT decryption of a 100 MiB uniform
random message split into 416,102 chunks of 252 bytes under 256 key pairs with
2048-bit moduli, chunk i under key i mod 256 -- the largest single-key-size
workload of the paper's file experiment (Sec. 4, Table 3: 2048-bit keys,
random files up to 100 MB).  Inputs are resident in HBM before timing starts.

Prints one JSON line:
  value  = 2048-bit CRT-decrypt modexps per second of whole steps (each step
           also encrypts every chunk, so this is a lower bound on the decrypt-only rate);
  roofline = the CRT-halves kernel (the dominant kernel) against the VALU
           integer multiply-add peak of the chip;
  cpu_baseline = the C oracle on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Canonical work of one Montgomery product with s 32-bit limbs (CIOS, Koc et al.
# 1996): 2 s^2 + s word products; exponentiation counts fixed at window 5.
def mm_products(s: int) -> int:
    return 2 * s * s + s


def half_products(bits: int) -> int:
    s_h = bits // 64
    W = -(-(bits // 2) // 5)
    return ((1 << 5) - 2 + (W - 1) * 6 + 2) * mm_products(s_h)


def crt_products(bits: int) -> int:
    s_h = bits // 64
    return 2 * half_products(bits) + 6 * mm_products(s_h) + s_h * s_h


def enc_products(bits: int, e: int = 65537) -> int:
    return ((e.bit_length() - 1) + (bin(e).count("1") - 1) + 2) * mm_products(bits // 32)


# Peak of the VALU 32x32->64 multiply-add (v_mad_u64_u32): one per lane per
# clock, 64 lanes per compute unit, 256 compute units, 2.4 GHz.
PEAK_MAD_PER_S = 256 * 64 * 2.4e9


def cpu_baseline(keys, msg, km, sample_chunks: int):
    import numpy as np

    import oracle

    n = min(sample_chunks, len(km))
    msg_s = msg[: n * 252]
    km_s = km[:n]
    table = oracle.KeyTable(keys)
    t0 = time.perf_counter()
    ct = oracle.encrypt(table, msg_s, km_s)
    t1 = time.perf_counter()
    pt, rc = oracle.decrypt(table, ct, len(msg_s), km_s, crt=True)
    t2 = time.perf_counter()
    assert rc == 0 and np.array_equal(pt, msg_s)
    return {
        "value": n / (t2 - t1),
        "unit": "2048-bit CRT decrypt modexp/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": f"first {n} chunks of the workload ({len(msg_s)} bytes, keys 0..{min(n, 256) - 1}): "
                  f"encrypt {t1 - t0:.2f} s, CRT decrypt {t2 - t1:.2f} s wall",
        "enc_MiBps": len(msg_s) / (t1 - t0) / 2**20,
        "dec_MiBps": len(msg_s) / (t2 - t1) / 2**20,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=1024, help="chunks the oracle baseline times")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--config", type=int, default=4,
                    help="workload recipe (1-4; the JSON line's headline workload is 4)")
    ap.add_argument("--mode", choices=["plain", "batch"], default="plain",
                    help="plain: per-class launches, each timed with HIP events during the timed steps; "
                         "batch: graph-captured batched path (kernel times from one extra profiled step)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(chunks are independent; see the sharding notes in DESIGN.md)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2111_11924_amd import binding, inputs

    w = inputs.config(args.config)
    keys, msg, km = w.keys(), w.message(), w.key_map()
    bits_of = np.array([k.bits for k in keys])[km]
    nchunks = len(km)
    ctx = binding.Context(0)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    d_msg = torch.from_numpy(msg).to("cuda")
    d_ct = torch.empty(plan.ct_len, dtype=torch.uint8, device="cuda")
    d_pt = torch.empty(len(msg), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    batch = args.mode == "batch"
    for _ in range(args.warmup):
        plan.encrypt(d_msg, d_ct, stream, batch=batch)
        plan.decrypt(d_ct, d_pt, stream, batch=batch)
    torch.cuda.synchronize()
    if args.warmup > 0 and (plan.check(stream) != binding.PMK_OK or not torch.equal(d_pt, d_msg)):
        print("warm-up output wrong: decrypt(encrypt(m)) != m", file=sys.stderr)
        return 1

    # plain mode: every launch of the timed steps is bracketed by HIP events on
    # the launch stream; batch mode replays the captured graphs untouched and
    # takes kernel times from one more (uncaptured, profiled) step afterwards
    plan.profile(not batch)
    marks = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        marks[k][0].record(stream)
        plan.encrypt(d_msg, d_ct, stream, batch=batch)
        marks[k][1].record(stream)
        plan.decrypt(d_ct, d_pt, stream, batch=batch)
        marks[k][2].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    enc_ms = sum(m[0].elapsed_time(m[1]) for m in marks)
    dec_ms = sum(m[1].elapsed_time(m[2]) for m in marks)
    ok = plan.check(stream) == binding.PMK_OK and torch.equal(d_pt, d_msg)
    prof_steps = args.steps
    if batch:
        plan.profile(True)
        plan.encrypt(d_msg, d_ct, stream, batch=True)
        plan.decrypt(d_ct, d_pt, stream, batch=True)
        torch.cuda.synchronize()
        prof_steps = 1

    halves_ms, halves_n = plan.kernel_time(binding.PMK_KERNEL_CRT_HALVES)
    kern = {binding.KERNEL_NAMES[k]: plan.kernel_time(k) for k in binding.KERNEL_NAMES}
    plan.profile(False)
    # algorithmic products of all CRT-halves launches in one step, over their time
    ub, uc = np.unique(bits_of, return_counts=True)
    # in batch mode the 3072/4096-bit classes run in the batch kernel instead
    halves_work = sum(2 * half_products(int(b)) * int(c) for b, c in zip(ub, uc)
                      if not (batch and int(b) > 2048))
    halves_avg_s = halves_ms / max(prof_steps, 1) / 1e3
    achieved = halves_work / halves_avg_s

    wall_s = t1 - t0
    ms_per_step = wall_s * 1e3 / args.steps
    mib = len(msg) / 2**20
    out = {
        "metric": "2048-bit CRT decrypt modexp/s + enc/dec MB/s on 1 MI355X; p99 request latency",
        "value": nchunks * args.steps / wall_s,
        "unit": "2048-bit CRT decrypt modexp/s (whole encrypt+decrypt steps)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w.name, "message_bytes": len(msg), "chunks": nchunks, "keys": len(keys),
                   "modulus_bits": sorted(set(int(k.bits) for k in keys)), "key_map": w.map_kind,
                   "public_exponent": 65537},
        "dec_modexp_per_s": nchunks * args.steps / (dec_ms / 1e3),
        "enc_modexp_per_s": nchunks * args.steps / (enc_ms / 1e3),
        "dec_MiBps": mib * args.steps / (dec_ms / 1e3),
        "enc_MiBps": mib * args.steps / (enc_ms / 1e3),
        "enc_ms_per_step": enc_ms / args.steps,
        "dec_ms_per_step": dec_ms / args.steps,
        "mode": args.mode,
        "kernel_ms_per_step": {k: v[0] / max(prof_steps, 1) for k, v in kern.items()},
        "roundtrip_ok": bool(ok),
        "p99_request_ms": None,
        "roofline": {
            "bound": "alu",
            "kernel": "crt_halves",
            "achieved": achieved / 1e12,
            "peak": PEAK_MAD_PER_S / 1e12,
            "unit": "Tmad/s (32x32->64 integer multiply-add)",
            "frac": achieved / PEAK_MAD_PER_S,
            "traffic": None,
            "work_per_step": halves_work,
            "avg_launch_ms": halves_ms / max(halves_n, 1),
            "launches_per_step": halves_n / max(prof_steps, 1),
        },
        "paper_context": {"table3_100MB_dec_s": 0.0622, "table3_100MB_enc_s": 0.0009,
                          "hardware": "NVIDIA P100 + Xeon Silver 4114 (context only)"},
    }
    if args.config != 4:
        out["metric"] = f"CRT decrypt modexp/s, workload {w.name}"
        out["unit"] = "CRT decrypt modexp/s (whole encrypt+decrypt steps)"
    if not args.no_cpu_baseline and args.config == 4:
        out["cpu_baseline"] = cpu_baseline(keys, msg, km, args.cpu_sample)
    plan.close()
    ctx.close()
    print(json.dumps(out))
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
