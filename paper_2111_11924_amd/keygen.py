"""Key generation with the primality tests on the GPU (pmk_sieve, pmk_miller_rabin).

The step before the encryption path: the key pairs of Algorithm 1's
initialisation (Sec. 1.1 step 1; Sec. 3.1).  Candidates and Miller-Rabin bases
are drawn on the host from a seeded PCG64 stream; trial division and the
Miller-Rabin rounds run on the GPU, one lane per candidate; the survivors are
paired into keys on the host (N = p q, d = e^-1 mod lcm(p-1, q-1), CRT
exponents and q^-1 mod p), as ``inputs.key_from_primes`` does.  Readings as in
``inputs``: primes of bits/2 bits with their top two bits set (so N has
exactly ``bits`` bits), gcd(e, p-1) = 1, p != q.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np

from . import binding, inputs


def _words(x: int, n: int) -> np.ndarray:
    return np.frombuffer(int(x).to_bytes(4 * n, "little"), dtype=np.uint32)


def gpu_primes(ctx: "binding.Context", bits: int, count: int, seed: int, rounds: int = 40,
               batch: int = 8192, e: int = inputs.E_DEFAULT) -> List[int]:
    """`count` distinct probable primes of bits/2 bits for `bits`-bit keys."""
    import torch

    half, words = bits // 2, bits // 64
    rng = np.random.Generator(np.random.PCG64(seed * 1000 + 6))
    found: List[int] = []
    seen = set()
    while len(found) < count:
        raw = rng.integers(0, 1 << 32, size=(batch, words), dtype=np.uint64).astype(np.uint32)
        raw[:, 0] |= 1                                   # odd
        raw[:, -1] |= np.uint32(3 << 30)                 # top two bits set
        d_cand = torch.from_numpy(raw.reshape(-1)).to("cuda")
        d_flags = torch.zeros(batch, dtype=torch.int32, device="cuda")
        binding.pmk_sieve(ctx.handle, bits, d_cand, batch, d_flags)
        keep = np.nonzero(d_flags.cpu().numpy())[0]
        cands = [int.from_bytes(raw[i].tobytes(), "little") for i in keep.tolist()]
        cands = [m for m in cands if math.gcd(e, m - 1) == 1 and m not in seen]
        if not cands:
            continue
        bases = np.zeros((len(cands), rounds, words), dtype=np.uint32)
        for i, m in enumerate(cands):
            for r in range(rounds):
                a = 2 + inputs.rand_int(rng, half + 64) % (m - 3)
                bases[i, r] = _words(a, words)
        packed = np.stack([_words(m, words) for m in cands])
        d_c = torch.from_numpy(packed.reshape(-1)).to("cuda")
        d_b = torch.from_numpy(bases.reshape(-1)).to("cuda")
        d_r = torch.zeros(len(cands), dtype=torch.int32, device="cuda")
        binding.pmk_miller_rabin(ctx.handle, bits, d_c, len(cands), d_b, rounds, d_r)
        res = d_r.cpu().numpy()
        for m, ok in zip(cands, res.tolist()):
            if ok and m not in seen:
                seen.add(m)
                found.append(m)
    return found[:count]


def gpu_make_keys(ctx: "binding.Context", bits: int, count: int, seed: int, rounds: int = 40) -> List[inputs.RsaKey]:
    """`count` RSA key pairs of `bits` bits (1024, 2048, 3072 or 4096) whose
    primes were found by the GPU primality tests."""
    primes = gpu_primes(ctx, bits, 2 * count, seed, rounds)
    keys = []
    for k in range(count):
        p, q = primes[2 * k], primes[2 * k + 1]
        key = inputs.key_from_primes(p, q, bits=bits)
        assert key.n.bit_length() == bits
        keys.append(key)
    return keys
