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


def _bases(rng: np.random.Generator, count: int, rounds: int, words: int) -> np.ndarray:
    """Random bases 1 < a < m - 1 for candidates whose top word is at least
    2^31 (top two bits set): a's top word is below 2^31, and a = 0 or 1 is
    replaced by 2."""
    a = rng.integers(0, 1 << 32, size=(count, rounds, words), dtype=np.uint64).astype(np.uint32)
    a[:, :, -1] &= np.uint32(0x7FFFFFFF)
    tiny = (a[:, :, 1:] == 0).all(axis=2) & (a[:, :, 0] < 2)
    a[:, :, 0][tiny] = 2
    return a


def gpu_primes(ctx: "binding.Context", bits: int, count: int, seed: int, rounds: int = 40,
               batch: int = 16384, e: int = inputs.E_DEFAULT) -> List[int]:
    """`count` distinct probable primes of bits/2 bits for `bits`-bit keys:
    GPU trial division, then one Miller-Rabin round on every survivor and the
    remaining rounds on those that pass it."""
    import torch

    words = bits // 64
    rng = np.random.Generator(np.random.PCG64(seed * 1000 + 6))
    found: List[int] = []
    seen = set()

    def mr(packed: np.ndarray, r: int) -> np.ndarray:
        d_c = torch.from_numpy(np.ascontiguousarray(packed).reshape(-1)).to("cuda")
        d_b = torch.from_numpy(_bases(rng, len(packed), r, words).reshape(-1)).to("cuda")
        d_r = torch.zeros(len(packed), dtype=torch.int32, device="cuda")
        binding.pmk_miller_rabin(ctx.handle, bits, d_c, len(packed), d_b, r, d_r)
        return d_r.cpu().numpy().astype(bool)

    while len(found) < count:
        raw = rng.integers(0, 1 << 32, size=(batch, words), dtype=np.uint64).astype(np.uint32)
        raw[:, 0] |= 1                                   # odd
        raw[:, -1] |= np.uint32(3 << 30)                 # top two bits set
        d_cand = torch.from_numpy(raw.reshape(-1)).to("cuda")
        d_flags = torch.zeros(batch, dtype=torch.int32, device="cuda")
        binding.pmk_sieve(ctx.handle, bits, d_cand, batch, d_flags)
        surv = raw[d_flags.cpu().numpy().astype(bool)]
        if len(surv) == 0:
            continue
        surv = surv[mr(surv, 1)]                         # one round weeds out the composites
        if len(surv) == 0:
            continue
        if rounds > 1:
            surv = surv[mr(surv, rounds - 1)]
        for row in surv:
            m = int.from_bytes(row.tobytes(), "little")
            if math.gcd(e, m - 1) == 1 and m not in seen:
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
