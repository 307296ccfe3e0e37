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


def joint_products(bits: int) -> int:
    """Canonical products of one prime's blinded decryption in one chain,
    (c*)^dp c_R^(p-1-dp) mod p, counted like half_products at window 5: both
    inputs reduced into Montgomery form and tabled (2 x 30 products), one
    squaring chain of 5 (W - 1) squarings with a window product for each of the
    two exponents per 5 bits, the c_R mod p check and the final conversion."""
    s_h = bits // 64
    W = -(-(bits // 2) // 5)
    return (2 * 30 + 4 + 5 * (W - 1) + 2 * (W - 1) + 1) * mm_products(s_h)


# Peak of the VALU 32x32->64 multiply-add (v_mad_u64_u32): one per lane per
# clock, 64 lanes per compute unit, 256 compute units, 2.4 GHz.
PEAK_MAD_PER_S = 256 * 64 * 2.4e9

# HBM traffic of the CRT-halves stage on the 100 MiB workload (halves_kernel
# over four full rounds, then the partial round as a launch of its own), from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) of
# `bench.py --no-serve --no-cpu-baseline --no-e2e --no-blinded --steps 2
# --warmup 1`, each scaled by what the counter reads for a plain 256 MiB device
# copy (bench.py --copy-probe 256: FETCH_SIZE reads half the bytes moved,
# WRITE_SIZE all of them).  Valid only for the kernel sources it was measured
# on (hash below); reported as null otherwise.
HALVES_TRAFFIC = {"sources_sha256": "6dc85095754025e0cb24fe72a1850cca3b276b2a4fd01d1f2a91e91903da5cc9",
                  "fetch_bytes": 20_217_526_800, "write_bytes": 2_582_776_832}
KERNEL_SOURCES = ["paper_2111_11924_amd/csrc/kernels_impl.hpp", "paper_2111_11924_amd/csrc/mont.hpp",
                  "paper_2111_11924_amd/csrc/mont_lanes.hpp", "paper_2111_11924_amd/csrc/pmk_internal.hpp",
                  "paper_2111_11924_amd/csrc/kernels_class.inc", "paper_2111_11924_amd/csrc/k2048.hip",
                  "paper_2111_11924_amd/csrc/klanes.hip"]


def kernel_sources_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def cpu_baseline(keys, msg, km, sample_chunks: int):
    """The C oracle (schoolbook products, Knuth D remainders, CRT) on the host
    cores: all threads on the first `sample_chunks` chunks, one thread on an
    eighth of them."""
    import numpy as np

    import oracle

    def run(n):
        msg_s = msg[: n * 252]
        km_s = km[:n]
        t0 = time.perf_counter()
        ct = oracle.encrypt(table, msg_s, km_s)
        t1 = time.perf_counter()
        pt, rc = oracle.decrypt(table, ct, len(msg_s), km_s, crt=True)
        t2 = time.perf_counter()
        assert rc == 0 and np.array_equal(pt, msg_s)
        return len(msg_s), t1 - t0, t2 - t1

    table = oracle.KeyTable(keys)
    n = min(sample_chunks, len(km))
    threads = oracle.threads()
    nbytes, te, td = run(n)
    oracle.set_threads(1)
    n1 = max(1, n // 8)
    nbytes1, te1, td1 = run(n1)
    oracle.set_threads(threads)
    return {
        "value": n / td,
        "unit": "2048-bit CRT decrypt modexp/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {n} chunks of the workload ({nbytes} bytes, keys 0..{min(n, 256) - 1}) on {threads} "
                  f"threads: encrypt {te:.2f} s, CRT decrypt {td:.2f} s wall; first {n1} chunks on 1 thread: "
                  f"encrypt {te1:.2f} s, CRT decrypt {td1:.2f} s",
        "enc_modexp_per_s": n / te,
        "enc_MiBps": nbytes / te / 2**20,
        "dec_MiBps": nbytes / td / 2**20,
        "single_thread": {"dec_modexp_per_s": n1 / td1, "enc_modexp_per_s": n1 / te1,
                          "dec_MiBps": nbytes1 / td1 / 2**20, "enc_MiBps": nbytes1 / te1 / 2**20},
    }


def blinding_blocks(keys, km, seed: int):
    """Blinding blocks for a throughput pass: per chunk kb random bytes with the
    top byte zero, so r < 2^(bits-8) < N; r shares a prime with N with
    probability below 2^-1000 (the GPU would report PMK_EBLIND).  Vectorised
    stand-in for inputs.make_blinding, whose per-chunk gcd is too slow for
    400,000 chunks; the timing does not depend on the values."""
    import numpy as np

    kb = np.array([k.bits // 8 for k in keys])[km]
    g = np.random.Generator(np.random.PCG64(seed * 1000 + 5))
    blk = g.integers(0, 256, size=int(kb.sum()), dtype=np.uint8)
    starts = np.concatenate([[0], np.cumsum(kb)[:-1]])
    blk[starts] = 0
    return blk


def blinded_measure(plan, d_msg, keys, km, seed: int, steps: int, warmup: int):
    """Blinded PMKRSA (Sec. 3.1) over the whole workload: c* = (r m)^e and
    c_R = r^e, then m = (c*)^d (c_R^d)^-1 through one squaring chain per prime;
    event-timed per call on the current stream, the one-chain kernel timed per
    launch in one extra profiled step."""
    import numpy as np
    import torch

    from paper_2111_11924_amd import binding

    stream = torch.cuda.current_stream()
    d_r = torch.from_numpy(blinding_blocks(keys, km, seed)).to("cuda")
    n = plan.ct_len
    d_cs = torch.empty(n, dtype=torch.uint8, device="cuda")
    d_cr = torch.empty(n, dtype=torch.uint8, device="cuda")
    d_pt = torch.empty(plan.msg_len, dtype=torch.uint8, device="cuda")
    enc = lambda: binding.pmk_encrypt_blinded_plan(plan.handle, d_msg, d_r, d_cs, d_cr, stream, plan.ctx.handle)
    dec = lambda: binding.pmk_decrypt_blinded_plan(plan.handle, d_cs, d_cr, d_pt, stream, plan.ctx.handle)
    for _ in range(warmup):
        enc()
        dec()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    for k in range(steps):
        ev[k][0].record(stream)
        enc()
        ev[k][1].record(stream)
        dec()
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    enc_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    dec_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
    ok = plan.check(stream) == binding.PMK_OK and torch.equal(d_pt, d_msg)
    plan.profile(True)
    dec()
    torch.cuda.synchronize()
    joint_ms, joint_n = plan.kernel_time(binding.PMK_KERNEL_CRT_HALVES)
    plan.profile(False)
    bits_of = np.array([k.bits for k in keys])[km]
    ub, uc = np.unique(bits_of, return_counts=True)
    work = sum(2 * joint_products(int(b)) * int(c) for b, c in zip(ub, uc))
    mib = plan.msg_len / 2**20
    return {
        "enc_ms": enc_ms, "dec_ms": dec_ms, "enc_MiBps": mib / (enc_ms / 1e3), "dec_MiBps": mib / (dec_ms / 1e3),
        "dec_modexp_per_s": len(km) / (dec_ms / 1e3), "roundtrip_ok": bool(ok),
        "roofline": {"bound": "alu", "kernel": "crt_halves_joint (one chain per prime)",
                     "achieved": work / (joint_ms / max(joint_n, 1) / 1e3) / 1e12, "peak": PEAK_MAD_PER_S / 1e12,
                     "unit": "Tmad/s", "frac": work / (joint_ms / max(joint_n, 1) / 1e3) / PEAK_MAD_PER_S,
                     "work_per_launch": work, "avg_launch_ms": joint_ms / max(joint_n, 1)},
    }


def host_measure(plan, msg, reps: int = 3):
    """End-to-end rates through the host-buffer forms (pmk_encrypt_host /
    pmk_decrypt_host, default slicing): pinned host message in, pinned host
    ciphertext out, and back; wall-clocked per call."""
    import numpy as np
    import torch

    from paper_2111_11924_amd import binding

    h_msg = torch.from_numpy(msg).pin_memory()
    h_ct = torch.empty(plan.ct_len, dtype=torch.uint8).pin_memory()
    h_pt = torch.empty(len(msg), dtype=torch.uint8).pin_memory()
    ok = plan.encrypt_host(h_msg, h_ct) == binding.PMK_OK and plan.decrypt_host(h_ct, h_pt) == binding.PMK_OK
    te = td = 0.0
    for _ in range(reps):
        t0 = time.perf_counter()
        ok = ok and plan.encrypt_host(h_msg, h_ct) == binding.PMK_OK
        t1 = time.perf_counter()
        ok = ok and plan.decrypt_host(h_ct, h_pt) == binding.PMK_OK
        t2 = time.perf_counter()
        te += t1 - t0
        td += t2 - t1
    ok = ok and bool(np.array_equal(h_pt.numpy(), msg))
    mib = len(msg) / 2**20
    return {"enc_MiBps_e2e": mib * reps / te, "dec_MiBps_e2e": mib * reps / td, "enc_ms_e2e": te / reps * 1e3,
            "dec_ms_e2e": td / reps * 1e3, "reps": reps, "host_buffers": "pinned", "ok": ok}


def serve_measure(nreq: int, loads, seed: int = 5, staging_mib: int = 2048, round_chunks: int = 0,
                  pipeline_depth: int = 0):
    """Serving workload: a 512-key device table (1024..4096-bit keys), requests
    of 1 KiB-10 MiB (log-uniform) over 1-64 keys each, half encryptions and
    half CRT decryptions.  First the closed-loop capacity (all requests queued
    at once), then Poisson arrivals at each fraction of it in `loads`; latency
    = completion (result in host memory) - scheduled arrival."""
    import numpy as np

    from paper_2111_11924_amd import binding, inputs

    w = inputs.config(5)
    keys = w.keys()
    bits = [int(k.bits) for k in keys]
    reqs = inputs.serving_requests(nreq, bits, seed)
    msgs = [r.message() for r in reqs]
    ctx = binding.Context(0)
    ctx.load_keys(keys)
    srv = ctx.server(staging_bytes=staging_mib << 20, round_chunks=round_chunks, pipeline_depth=pipeline_depth)
    try:
        # ciphertexts of the decryption requests, made outside any timing
        pend = [(i, srv.submit(binding.PMK_OP_ENCRYPT, msgs[i], len(msgs[i]), r.key_map))
                for i, r in enumerate(reqs) if r.op == binding.PMK_OP_DECRYPT]
        cts = {}
        for i, (t, out) in pend:
            assert srv.wait(t)["status"] == binding.PMK_OK
            cts[i] = out
        data = [cts[i] if r.op == binding.PMK_OP_DECRYPT else msgs[i] for i, r in enumerate(reqs)]

        def run(offsets):
            t0 = time.monotonic_ns() + 2_000_000
            tickets = []
            for i, r in enumerate(reqs):
                due = t0 + (int(offsets[i] * 1e9) if offsets is not None else 0)
                while True:
                    now = time.monotonic_ns()
                    if now >= due:
                        break
                    time.sleep(min((due - now) / 1e9, 0.002))
                tickets.append((due, srv.submit(r.op, data[i], len(msgs[i]), r.key_map)))
            lat, ok = [], True
            t_end = t0
            for i, (due, (t, out)) in enumerate(tickets):
                info = srv.wait(t)
                ok = ok and info["status"] == binding.PMK_OK
                if reqs[i].op == binding.PMK_OP_DECRYPT:
                    ok = ok and np.array_equal(out, msgs[i])
                lat.append((info["t_done_ns"] - due) / 1e6)
                t_end = max(t_end, info["t_done_ns"])
            return np.array(lat), (t_end - t0) / 1e9, ok

        lat, wall, ok = run(None)
        cap = nreq / wall
        nbytes = sum(len(m) for m in msgs)
        out = {"requests": nreq, "mean_request_bytes": nbytes / nreq,
               "capacity_req_per_s": cap, "capacity_MiBps": nbytes / wall / 2**20, "results_ok": bool(ok),
               "points": []}
        for f in loads:
            arr = inputs.poisson_arrivals(nreq, f * cap, seed)
            lat, wall, ok2 = run(arr)
            out["results_ok"] = out["results_ok"] and bool(ok2)
            out["points"].append({"load": f, "rate_req_per_s": f * cap, "p50_ms": float(np.percentile(lat, 50)),
                                  "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
                                  "achieved_req_per_s": nreq / wall})
        out["server_stats"] = srv.stats()
    finally:
        srv.stop()
        ctx.close()
    return out


# The paper's Table 2, configuration D (P100 + Xeon, 16 keys, 100 KB): seconds
PAPER_TABLE2_D = {2048: (0.0009, 0.0611), 3072: (0.0014, 0.1419), 4096: (0.0021, 0.2763),
                  6144: (0.0036, 0.7873), 8192: (0.0060, 1.6665)}


def paper_table(steps: int, warmup: int):
    """Per-size experiment of the paper (Sec. 4, Tables 1-2): 100 KB under 16
    keys of each size, plain RSA chunks and blinded PMKRSA chunks, device-resident,
    event-timed per call; the paper's configuration-D seconds beside them."""
    import numpy as np
    import torch

    from paper_2111_11924_amd import binding, inputs

    rows = []
    stream = torch.cuda.current_stream()
    for bits in inputs.TABLE_BITS:
        w = inputs.table_workload(bits)
        keys, msg, km = w.keys(), w.message(), w.key_map()
        ctx = binding.Context(0)
        ctx.load_keys(keys)
        plan = ctx.plan(km, len(msg))
        d_msg = torch.from_numpy(msg).to("cuda")
        d_r = torch.from_numpy(inputs.make_blinding(keys, km, w.seed)).to("cuda")
        d_ct = torch.empty(plan.ct_len, dtype=torch.uint8, device="cuda")
        d_cs = torch.empty(plan.ct_len, dtype=torch.uint8, device="cuda")
        d_cr = torch.empty(plan.ct_len, dtype=torch.uint8, device="cuda")
        d_pt = torch.empty(len(msg), dtype=torch.uint8, device="cuda")
        d_pb = torch.empty(len(msg), dtype=torch.uint8, device="cuda")
        ops = {
            "enc": lambda: binding.pmk_encrypt_plan(plan.handle, d_msg, d_ct, stream, ctx.handle),
            "dec": lambda: binding.pmk_decrypt_plan(plan.handle, d_ct, d_pt, stream, ctx.handle),
            "enc_blinded": lambda: binding.pmk_encrypt_blinded_plan(plan.handle, d_msg, d_r, d_cs, d_cr, stream,
                                                                    ctx.handle),
            "dec_blinded": lambda: binding.pmk_decrypt_blinded_plan(plan.handle, d_cs, d_cr, d_pb, stream,
                                                                    ctx.handle),
        }
        row = {"bits": bits, "keys": 16, "message_bytes": len(msg), "chunks": len(km)}
        for name, fn in ops.items():
            for _ in range(warmup):
                fn()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            torch.cuda.synchronize()
            ev[0].record(stream)
            for _ in range(steps):
                fn()
            ev[1].record(stream)
            torch.cuda.synchronize()
            row[name + "_s"] = ev[0].elapsed_time(ev[1]) / steps / 1e3
        row["ok"] = bool(plan.check(stream) == binding.PMK_OK and torch.equal(d_pt, d_msg)
                         and torch.equal(d_pb, d_msg))
        row["paper_D_enc_s"], row["paper_D_dec_s"] = PAPER_TABLE2_D[bits]
        rows.append(row)
        plan.close()
        ctx.close()
    return rows


def mp_products(bits: int) -> int:
    """Canonical word products of one multi-prime CRT decryption (bits/1024
    primes of 1024 bits): per prime one exponentiation by a 1024-bit exponent
    (the 2048-bit key's half count) plus the reduction of the input's remaining
    pieces, then the recombination's b(b-1)/2 products modulo the primes."""
    b = bits // 1024
    return b * (half_products(2048) + (b - 2) * mm_products(32)) + b * (b - 1) // 2 * mm_products(32)


def multi_prime_measure(steps: int, warmup: int, mib: int = 64):
    """Multi-prime CRT decryption (Sec. 2.1: b primes of bits/b bits) against
    two-prime CRT decryption of the same ciphertext under keys of the same
    size, both through their synchronous one-shot entry points (plan, run,
    check, free), wall-clocked per call.  Ciphertext: seeded random blocks
    below 2^(bits-8), device-resident; 4 keys per size, chunk i under key i mod 4."""
    import numpy as np
    import torch

    from paper_2111_11924_amd import binding, inputs

    rows = []
    for bits in (3072, 4096):
        mp_keys = [inputs.make_mp_key(bits, 77, i) for i in range(4)]
        two = inputs.make_keys([bits] * 4, 77)
        msg_len = mib << 20
        km = inputs.round_robin_map(msg_len, [bits] * 4)
        kb = bits // 8
        g = np.random.Generator(np.random.PCG64([77, bits]))
        ct = g.integers(0, 256, size=len(km) * kb, dtype=np.uint8)
        ct.reshape(-1, kb)[:, 0] = 0
        d_ct = torch.from_numpy(ct).to("cuda")
        d_mp = torch.empty(msg_len, dtype=torch.uint8, device="cuda")
        d_2p = torch.empty(msg_len, dtype=torch.uint8, device="cuda")
        ctx = binding.Context(0)
        ctx.load_mp_keys(mp_keys)
        ctx.load_keys(two)
        calls = {
            "multi_prime": lambda: binding.pmk_mp_decrypt(ctx.handle, d_ct, len(ct), km, d_mp, msg_len),
            "two_prime": lambda: binding.pmk_decrypt(ctx.handle, d_ct, len(ct), km, d_2p, msg_len),
        }
        row = {"bits": bits, "primes": bits // 1024, "keys": 4, "message_bytes": msg_len, "chunks": len(km)}
        ok = True
        for name, fn in calls.items():
            for _ in range(warmup):
                ok &= fn() == binding.PMK_OK
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                ok &= fn() == binding.PMK_OK
            torch.cuda.synchronize()
            row[name + "_ms"] = (time.perf_counter() - t0) / steps * 1e3
            row[name + "_chunks_per_s"] = len(km) / row[name + "_ms"] * 1e3
        row["speedup"] = row["two_prime_ms"] / row["multi_prime_ms"]
        row["model_speedup"] = (bits // 1024) ** 2 / 4
        row["mp_mad_frac_wall"] = len(km) * mp_products(bits) / (row["multi_prime_ms"] / 1e3) / PEAK_MAD_PER_S
        row["ok"] = bool(ok)
        rows.append(row)
        ctx.close()
    return rows


def keygen_measure(bits: int, count: int, rounds: int, seed: int = 950):
    """Key generation with the GPU primality tests (sieve + Miller-Rabin) against
    the host's own search (inputs.gen_prime: numpy sieve + Python pow) on a
    bounded sample."""
    import numpy as np

    from paper_2111_11924_amd import binding, inputs, keygen

    ctx = binding.Context(0)
    ctx.load_keys(inputs.make_keys([1024], 900))
    keygen.gpu_make_keys(ctx, bits, 2, seed + 1, rounds)  # warm-up
    t0 = time.perf_counter()
    keys = keygen.gpu_make_keys(ctx, bits, count, seed, rounds)
    t1 = time.perf_counter()
    ok = all(binding.pmk_key_check(k)[0] == binding.PMK_OK for k in keys)
    ctx.close()
    g = np.random.Generator(np.random.PCG64(seed))
    n_host = 4
    t2 = time.perf_counter()
    for _ in range(n_host):
        inputs.gen_prime(bits // 2, g)
    t3 = time.perf_counter()
    return {"bits": bits, "keys": count, "rounds": rounds, "gpu_s": t1 - t0, "gpu_keys_per_s": count / (t1 - t0),
            "host_primes": n_host, "host_s": t3 - t2, "host_keys_per_s": n_host / 2 / (t3 - t2), "keys_ok": ok}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=2048, help="chunks the oracle baseline times")
    ap.add_argument("--autotune", action="store_true",
                    help="pick each class's CRT window by timing on this device first (pmk_autotune)")
    ap.add_argument("--window", type=int, default=0, help="fix the CRT window width of every class")
    ap.add_argument("--lanes", type=int, nargs=2, default=None, metavar=("FILL", "TAIL"),
                    help="lanes per number (1, 2, 4) of the CRT halves of an under-filled launch and of a "
                         "short last round, every one-lane class")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the short serving pass that fills p99_request_ms")
    ap.add_argument("--paper-table", action="store_true",
                    help="the paper's per-size experiment: 100 KB under 16 keys of 2048..8192 bits")
    ap.add_argument("--keygen", action="store_true",
                    help="key generation with the GPU primality tests (2048-bit keys)")
    ap.add_argument("--multi-prime", action="store_true",
                    help="multi-prime CRT decryption (3072/3 and 4096/4 primes) against two-prime CRT")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload only: capacity, then Poisson loads 0.5/0.8/1.2 of it")
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="requests per serving point (default: 2000 with --serve, 300 for the headline p99)")
    ap.add_argument("--round-chunks", type=int, default=0,
                    help="server: most chunks per batching round (0: the library default)")
    ap.add_argument("--pipeline-depth", type=int, default=0, help="server: rounds in flight (1 or 2)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates HBM byte counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-blinded", action="store_true", help="skip the blinded PMKRSA pass after the timed steps")
    ap.add_argument("--no-e2e", action="store_true", help="skip the end-to-end pass through host buffers")
    ap.add_argument("--config", type=int, default=4,
                    help="workload recipe (1-4; the JSON line's headline workload is 4)")
    ap.add_argument("--mode", choices=["plain", "batch"], default="plain",
                    help="plain: per-class launches, each timed with HIP events during the timed steps; "
                         "batch: graph-captured batched path (kernel times from one extra profiled step)")
    ap.add_argument("--lib", default=None, metavar="PATH",
                    help="load this build of libpmk.so instead of the package's own (A/B of two builds)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (chunks are independent, so "
              "each GPU would take its own slice of the chunk range with a copy of the key table)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2111_11924_amd import binding, inputs

    if args.lib:
        binding.LIB_PATH = os.path.abspath(args.lib)
    if args.serve:
        res = serve_measure(args.serve_requests or 2000, [0.5, 0.8, 1.2], round_chunks=args.round_chunks,
                            pipeline_depth=args.pipeline_depth)
        res["round_chunks"] = args.round_chunks
        res["pipeline_depth"] = args.pipeline_depth
        res.update({"metric": "p99 request latency, serving workload (512 keys, 1 KiB-10 MiB requests)",
                    "unit": "ms", "n_gpus": 1, "data": "synthetic", "higher_is_better": False,
                    "value": res["points"][1]["p99_ms"], "config": {"workload": "serving-512keys-mixed",
                                                                    "load_for_value": 0.8}})
        print(json.dumps(res))
        return 0 if res["results_ok"] else 1

    if args.keygen:
        res = keygen_measure(2048, 64, 40)
        res.update({"metric": "2048-bit RSA key pairs per second (GPU sieve + 40 Miller-Rabin rounds)",
                    "unit": "keys/s", "value": res["gpu_keys_per_s"], "n_gpus": 1, "data": "synthetic",
                    "higher_is_better": True, "config": {"workload": "keygen-2048b"}})
        print(json.dumps(res))
        return 0 if res["keys_ok"] else 1

    if args.multi_prime:
        rows = multi_prime_measure(args.steps, args.warmup)
        print(json.dumps({"metric": "multi-prime CRT decryption, chunks per second (one-shot calls)",
                          "unit": "chunks/s", "n_gpus": 1, "data": "synthetic", "higher_is_better": True,
                          "value": rows[-1]["multi_prime_chunks_per_s"],
                          "config": {"workload": "mp-64MiB-4keys", "key_bits": [r["bits"] for r in rows]},
                          "rows": rows}))
        return 0 if all(r["ok"] for r in rows) else 1

    if args.paper_table:
        rows = paper_table(args.steps, args.warmup)
        print(json.dumps({"metric": "seconds per 100 KB, encrypt / CRT decrypt, plain and blinded PMKRSA chunks",
                          "unit": "s", "n_gpus": 1, "data": "synthetic", "higher_is_better": False,
                          "config": {"workload": "table-100KB-16keys", "key_bits": [r["bits"] for r in rows]},
                          "rows": rows,
                          "paper_context": "paper Table 2, configuration D: NVIDIA P100 + Xeon, context only"}))
        return 0 if all(r["ok"] for r in rows) else 1

    if args.copy_probe:
        # a copy of known size: what FETCH_SIZE / WRITE_SIZE read for it scales
        # the same counters taken over the path's kernels
        n = args.copy_probe << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "copies": 3}))
        return 0

    w = inputs.config(args.config)
    keys, msg, km = w.keys(), w.message(), w.key_map()
    bits_of = np.array([k.bits for k in keys])[km]
    nchunks = len(km)
    ctx = binding.Context(0)
    ctx.load_keys(keys)
    if args.window:
        for b in set(int(k.bits) for k in keys):
            ctx.set_window(b, args.window)
    elif args.autotune:
        ctx.autotune()  # measured on this device (setup, outside the timed region)
    if args.lanes:
        for b in set(int(k.bits) for k in keys):
            if b <= 4096:
                ctx.set_lanes(b, args.lanes[0], args.lanes[1])
    windows = {int(b): ctx.window(int(b)) for b in sorted(set(int(k.bits) for k in keys))}
    lanes = {int(b): ctx.lanes(int(b)) for b in sorted(set(int(k.bits) for k in keys))}
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
    step_ms = sorted(m[0].elapsed_time(m[2]) for m in marks)
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
    halves_work = sum(2 * half_products(int(b)) * int(c) for b, c in zip(ub, uc))
    # plain mode: the CRT-halves launches run one after another, so their
    # summed event times are the stage's time; batch mode runs them side by
    # side, so the whole decryption pass (event-timed per step) stands in
    halves_avg_s = (halves_ms / max(prof_steps, 1) if not batch else dec_ms / args.steps) / 1e3
    achieved = halves_work / halves_avg_s

    traffic = None
    if (args.config == 4 and args.window in (0, 5) and not args.autotune and not args.lib and HALVES_TRAFFIC["fetch_bytes"]
            and HALVES_TRAFFIC["sources_sha256"] == kernel_sources_sha256()):
        traffic = HALVES_TRAFFIC["fetch_bytes"] + HALVES_TRAFFIC["write_bytes"]
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
        "crt_window": windows,
        "tail_lanes": lanes,
        "step_ms_median": step_ms[len(step_ms) // 2],
        "step_ms_min": step_ms[0],
        "half_modexp_per_s": 2 * nchunks * args.steps / (dec_ms / 1e3),
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
            "traffic": traffic,
            "work_per_step": halves_work,
            "avg_launch_ms": halves_ms / max(halves_n, 1),
            "stage_ms_per_step": halves_avg_s * 1e3,
            "launches_per_step": halves_n / max(prof_steps, 1),
        },
        "paper_context": {"table3_100MB_dec_s": 0.0622, "table3_100MB_enc_s": 0.0009,
                          "hardware": "NVIDIA P100 + Xeon Silver 4114 (context only)"},
    }
    if args.config != 4:
        out["metric"] = f"CRT decrypt modexp/s, workload {w.name}"
        out["unit"] = "CRT decrypt modexp/s (whole encrypt+decrypt steps)"
    # after the timed region: end-to-end rates from pinned host memory, and
    # blinded PMKRSA over the same workload
    if not args.no_e2e:
        e2e = host_measure(plan, msg)
        out.update({k: v for k, v in e2e.items() if k.endswith("_e2e")})
        out["e2e"] = {"reps": e2e["reps"], "host_buffers": e2e["host_buffers"], "ok": e2e["ok"],
                      "form": "pmk_encrypt_host / pmk_decrypt_host (H2D, compute, D2H over slices)"}
        ok = ok and e2e["ok"]
    if not args.no_blinded and not batch:
        bl = blinded_measure(plan, d_msg, keys, km, w.seed, max(2, min(args.steps, 5)), 1)
        out["blinded"] = bl
        ok = ok and bl["roundtrip_ok"]
    plan.close()
    ctx.close()
    if not args.no_serve and args.config == 4:
        # serving workload after the timed region: p99 at 0.8 of capacity
        sv = serve_measure(args.serve_requests or 300, [0.8], round_chunks=args.round_chunks)
        out["p99_request_ms"] = sv["points"][0]["p99_ms"]
        out["serving"] = {"workload": "serving-512keys-mixed", "requests": sv["requests"],
                          "capacity_req_per_s": sv["capacity_req_per_s"], "capacity_MiBps": sv["capacity_MiBps"],
                          "load": 0.8, "p50_ms": sv["points"][0]["p50_ms"], "p99_ms": sv["points"][0]["p99_ms"],
                          "results_ok": sv["results_ok"]}
        ok = ok and sv["results_ok"]
    if not args.no_cpu_baseline and args.config == 4:
        out["cpu_baseline"] = cpu_baseline(keys, msg, km, args.cpu_sample)
    print(json.dumps(out))
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
