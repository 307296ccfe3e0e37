"""Seeded synthetic inputs: RSA key pairs, random messages and chunk-to-key maps.

This module produces inputs only.  It holds none of the encryption or decryption
arithmetic: key generation uses Python's built-in integers (``pow`` for
Miller-Rabin and modular inverses), messages are uniform random bytes, as the
paper's test files are (Sec. 4, randomly generated files of 1-100 MB).

Key generation follows the standard RSA initialisation (Sec. 1.1, step 1;
Algorithm 1, Initialization): two distinct primes p, q of half the modulus
length, N = p q, public exponent e = 65537 (the Fermat number F_4 named in
Sec. 3.4), d = e^-1.  Readings taken where the paper is silent:

* d is the inverse of e modulo lambda(N) = lcm(p-1, q-1) (the paper writes phi;
  d_p, d_q and every decryption result are the same either way);
* both primes get their top two bits set, so N has exactly ``bits`` bits; p > q;
* randomness is a seeded PCG64 stream instead of /dev/random, so runs repeat.

Besides the textbook fields each key carries the two constants the GPU
library's key table takes with the modulus: ``n0inv = -N^-1 mod 2^32`` and
``rr = R^2 mod N`` with ``R = 2^bits``.

Workload recipes (the configurations the benchmarks and parity tests use) are in
``CONFIGS``; sub-seeds are ``seed*1000 + 1`` (keys), ``+2`` (message bytes),
``+3`` (chunk-to-key map), ``+4`` (arrivals).
"""
from __future__ import annotations

import hashlib
import json
import math
import os
from concurrent.futures import ProcessPoolExecutor
from dataclasses import dataclass, field
from multiprocessing import get_context
from typing import Dict, List, Optional, Sequence

import numpy as np

E_DEFAULT = 65537

_SMALL_PRIMES: Optional[np.ndarray] = None


def _small_primes(limit: int = 1 << 16) -> np.ndarray:
    global _SMALL_PRIMES
    if _SMALL_PRIMES is None:
        sieve = np.ones(limit, dtype=bool)
        sieve[:2] = False
        for i in range(2, int(limit ** 0.5) + 1):
            if sieve[i]:
                sieve[i * i :: i] = False
        _SMALL_PRIMES = np.nonzero(sieve)[0][1:].astype(np.int64)  # odd primes only
    return _SMALL_PRIMES


def rand_int(rng: np.random.Generator, nbits: int) -> int:
    """A uniform integer in [0, 2^nbits) drawn from ``rng``."""
    nwords = (nbits + 31) // 32
    words = rng.integers(0, 1 << 32, size=nwords, dtype=np.uint64)
    x = 0
    for w in words:
        x = (x << 32) | int(w)
    return x >> (32 * nwords - nbits)


def _mr_rounds(bits: int) -> int:
    # FIPS 186-4 style round counts for randomly searched candidates; tests
    # cross-check primality of generated keys with an independent routine.
    if bits >= 1536:
        return 4
    if bits >= 1024:
        return 5
    if bits >= 512:
        return 8
    if bits >= 256:
        return 16
    return 40


def is_probable_prime(n: int, rng: np.random.Generator, rounds: int) -> bool:
    """Miller-Rabin: base 2 first, then ``rounds - 1`` random bases."""
    if n < 4:
        return n in (2, 3)
    if n % 2 == 0:
        return False
    for sp in (3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % sp == 0:
            return n == sp
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    bases = [2] + [2 + rand_int(rng, n.bit_length() + 8) % (n - 3) for _ in range(rounds - 1)]
    for a in bases:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def gen_prime(bits: int, rng: np.random.Generator, e: int = E_DEFAULT) -> int:
    """A probable prime of exactly ``bits`` bits with its top two bits set and
    gcd(e, p-1) = 1: incremental search from a random odd start, sieved by the
    odd primes below 2^16."""
    if bits < 8:
        raise ValueError("prime size too small")
    primes = _small_primes()
    window = 4096 if bits < 1024 else 8192
    while True:
        start = rand_int(rng, bits) | (3 << (bits - 2)) | 1
        keep = np.ones(window, dtype=bool)  # candidate start + 2k
        ps = primes[primes < start]
        rem = np.array([start % int(p) for p in ps], dtype=np.int64)
        inv2 = (ps + 1) // 2
        first = ((ps - rem) % ps) * inv2 % ps
        for p, k0 in zip(ps.tolist(), first.tolist()):
            keep[k0::p] = False
        for k in np.nonzero(keep)[0].tolist():
            cand = start + 2 * k
            if cand.bit_length() != bits:
                break
            if math.gcd(e, cand - 1) != 1:
                continue
            if is_probable_prime(cand, rng, _mr_rounds(bits)):
                return cand


@dataclass
class RsaKey:
    """One key pair; every field a Python int (``bits`` = modulus length)."""

    bits: int
    n: int
    e: int
    d: int
    p: int
    q: int
    dp: int
    dq: int
    qinv: int
    n0inv: int
    rr: int

    def to_json(self) -> dict:
        return {k: (hex(v) if k != "bits" else v) for k, v in self.__dict__.items()}

    @staticmethod
    def from_json(obj: dict) -> "RsaKey":
        return RsaKey(**{k: (int(v, 16) if k != "bits" else int(v)) for k, v in obj.items()})


def key_from_primes(p: int, q: int, e: int = E_DEFAULT, bits: Optional[int] = None,
                    use_lambda: bool = True) -> RsaKey:
    """Complete a key pair from its primes (Sec. 1.1 step 1; p > q after swap)."""
    if p < q:
        p, q = q, p
    n = p * q
    if bits is None:
        bits = n.bit_length()
    phi = (p - 1) * (q - 1)
    lam = phi // math.gcd(p - 1, q - 1)
    d = pow(e, -1, lam if use_lambda else phi)
    rr = pow(2, 2 * bits, n)
    n0inv = (-pow(n, -1, 1 << 32)) % (1 << 32) if n % 2 else 0
    return RsaKey(bits=bits, n=n, e=e, d=d, p=p, q=q, dp=d % (p - 1), dq=d % (q - 1),
                  qinv=pow(q, -1, p), n0inv=n0inv, rr=rr)


def make_key(bits: int, seed: int, index: int, e: int = E_DEFAULT) -> RsaKey:
    """Key ``index`` of the seeded stream ``seed`` with a ``bits``-bit modulus."""
    if bits % 64 or bits < 128:
        raise ValueError("modulus bits must be a multiple of 64, at least 128")
    rng = np.random.Generator(np.random.PCG64([seed, index, bits]))
    half = bits // 2
    p = gen_prime(half, rng, e)
    while True:
        q = gen_prime(half, rng, e)
        if q != p:
            break
    key = key_from_primes(p, q, e, bits)
    assert key.n.bit_length() == bits
    return key


@dataclass
class MpKey:
    """A multi-prime key (Sec. 2.1, multi-prime variant): N = p_0 ... p_(b-1);
    ``exps`` holds d_i = d mod (p_i - 1).  ``p, q, dp, dq, qinv`` are zero (no
    two-prime split), so the oracle's plain c^d route is the one that applies."""

    bits: int
    n: int
    e: int
    d: int
    primes: List[int]
    exps: List[int]
    p: int = 0
    q: int = 0
    dp: int = 0
    dq: int = 0
    qinv: int = 0


def make_mp_key(bits: int, seed: int, index: int, e: int = E_DEFAULT) -> MpKey:
    """Multi-prime key ``index`` of stream ``seed``: bits/1024 distinct primes of
    1024 bits (3072 bits: 3 primes, 4096 bits: 4); d = e^-1 mod lcm(p_i - 1)."""
    if bits not in (3072, 4096):
        raise ValueError("multi-prime keys are 3072 or 4096 bits")
    rng = np.random.Generator(np.random.PCG64([seed, index, bits, 7]))
    primes: List[int] = []
    while True:
        while len(primes) < bits // 1024:
            p = gen_prime(1024, rng, e)
            if p not in primes:
                primes.append(p)
        n = math.prod(primes)
        if n.bit_length() == bits:
            break
        primes.remove(min(primes))  # product one bit short: redraw its smallest prime
    lam = 1
    for p in primes:
        lam = lam * (p - 1) // math.gcd(lam, p - 1)
    d = pow(e, -1, lam)
    return MpKey(bits=bits, n=n, e=e, d=d, primes=primes, exps=[d % (p - 1) for p in primes])


def _make_key_args(args):
    return make_key(*args).to_json()


def _cache_dir() -> str:
    root = os.environ.get("PMK_KEYCACHE")
    if root:
        return root
    return os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "_build",
                        "keycache")


def make_keys(bits_list: Sequence[int], seed: int, e: int = E_DEFAULT,
              workers: Optional[int] = None, cache: bool = True) -> List[RsaKey]:
    """Keys 0..len(bits_list)-1 of stream ``seed``, key j with bits_list[j] bits.

    Deterministic in its arguments; cached on disk (``_build/keycache``, or
    ``$PMK_KEYCACHE``) because large keys take seconds each to generate.  Large
    sets are generated by a pool of child processes (started fresh, not forked).
    """
    bits_list = [int(b) for b in bits_list]
    tag = hashlib.sha256(json.dumps([bits_list, seed, e]).encode()).hexdigest()[:20]
    path = os.path.join(_cache_dir(), f"keys_{tag}.json")
    if cache and os.path.exists(path):
        try:
            with open(path) as f:
                return [RsaKey.from_json(o) for o in json.load(f)]
        except (OSError, ValueError):
            pass
    jobs = [(b, seed, j, e) for j, b in enumerate(bits_list)]
    cost = sum((b / 1024.0) ** 3 for b in bits_list)
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers > 1 and cost > 8:
        with ProcessPoolExecutor(max_workers=workers, mp_context=get_context("spawn")) as ex:
            objs = list(ex.map(_make_key_args, jobs, chunksize=1))
    else:
        objs = [_make_key_args(j) for j in jobs]
    if cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = f"{path}.{os.getpid()}.tmp"
            with open(tmp, "w") as f:
                json.dump(objs, f)
            os.replace(tmp, path)
        except OSError:
            pass
    return [RsaKey.from_json(o) for o in objs]


def make_message(nbytes: int, seed: int) -> np.ndarray:
    """``nbytes`` uniform random bytes (uint8 array) from sub-seed seed*1000+2."""
    rng = np.random.Generator(np.random.PCG64(seed * 1000 + 2))
    return rng.integers(0, 256, size=nbytes, dtype=np.uint8)


def round_robin_map(msg_len: int, key_bits: Sequence[int]) -> np.ndarray:
    """Chunk i under key i mod K; as many chunks as the message needs.  Chunk i
    carries (bits/8 - 4) bytes of its key, the last chunk the remainder."""
    caps = [b // 8 - 4 for b in key_bits]
    out = []
    left, i, K = msg_len, 0, len(key_bits)
    while left > 0:
        k = i % K
        out.append(k)
        left -= caps[k]
        i += 1
    return np.array(out, dtype=np.uint32)


def random_map(msg_len: int, key_bits: Sequence[int], seed: int) -> np.ndarray:
    """Chunk keys drawn uniformly (sub-seed seed*1000+3), one chunk at a time,
    until the message is consumed."""
    rng = np.random.Generator(np.random.PCG64(seed * 1000 + 3))
    caps = np.array([b // 8 - 4 for b in key_bits], dtype=np.int64)
    out: List[int] = []
    left = msg_len
    while left > 0:
        draw = rng.integers(0, len(key_bits), size=4096)
        for k in draw.tolist():
            if left <= 0:
                break
            out.append(k)
            left -= int(caps[k])
    return np.array(out, dtype=np.uint32)


MiB = 1 << 20


@dataclass
class Workload:
    """One configuration: key sizes, message length, map kind, seed."""

    name: str
    seed: int
    key_bits: List[int]
    msg_len: int
    map_kind: str  # "round_robin" | "random"
    notes: str = ""
    _keys: Optional[List[RsaKey]] = field(default=None, repr=False)

    def keys(self) -> List[RsaKey]:
        if self._keys is None:
            self._keys = make_keys(self.key_bits, self.seed * 1000 + 1)
        return self._keys

    def message(self) -> np.ndarray:
        return make_message(self.msg_len, self.seed)

    def key_map(self) -> np.ndarray:
        if self.map_kind == "round_robin":
            return round_robin_map(self.msg_len, self.key_bits)
        return random_map(self.msg_len, self.key_bits, self.seed)


def _mixed_bits(count: int, seed: int, choices=(1024, 2048, 3072, 4096)) -> List[int]:
    rng = np.random.Generator(np.random.PCG64(seed * 1000 + 5))
    return [int(choices[i]) for i in rng.integers(0, len(choices), size=count)]


def config(idx: int) -> Workload:
    """The five workload recipes (modulus bits, message bytes, map, seed)."""
    if idx == 1:
        return Workload("small-512b-16KiB", 1, [512] * 8, 16 * 1024, "round_robin",
                        "8 keys, 60-byte chunks, chunk i under key i mod 8")
    if idx == 2:
        return Workload("plain-2048b-1MiB", 2, [2048] * 64, 1 * MiB, "round_robin",
                        "64 keys, 252-byte chunks, round-robin")
    if idx == 3:
        return Workload("mixed-1024to4096b-25MiB", 3, _mixed_bits(256, 3), 25 * MiB, "random",
                        "256 keys of 1024/2048/3072/4096 bits, seeded random map")
    if idx == 4:
        return Workload("plain-2048b-100MiB", 4, [2048] * 256, 100 * MiB, "round_robin",
                        "256 keys, 252-byte chunks (416,102), round-robin")
    if idx == 5:
        return Workload("serving-512keys-mixed", 5, _mixed_bits(512, 5), 0, "per_request",
                        "512-key table, Poisson arrivals, 1 KiB-10 MiB requests")
    raise ValueError(idx)


# Key sizes of the paper's per-size experiment (Sec. 4, Tables 1 and 2).
TABLE_BITS = (2048, 3072, 4096, 6144, 8192)


def table_workload(bits: int) -> Workload:
    """The paper's per-size experiment (Sec. 4, Tables 1-2, configuration D):
    a 102,400-byte random plaintext under 16 key pairs of one size, chunk i
    under key i mod 16."""
    return Workload(f"table-{bits}b-100KB", 600 + bits // 64, [bits] * 16, 102_400, "round_robin",
                    "16 keys, 100 KB, round-robin")


CONFIGS: Dict[int, str] = {i: config(i).name for i in range(1, 6)}


def make_blinding(keys: Sequence["RsaKey"], key_map: np.ndarray, seed: int) -> np.ndarray:
    """Blinding factors of the PMKRSA scheme (Sec. 3.1): per chunk an r uniform
    in [2, N-1] with gcd(r, N) = 1 under the chunk's key, as kb-byte big-endian
    blocks laid out like the ciphertext (the scheme draws them; here they are
    seeded inputs)."""
    rng = np.random.Generator(np.random.PCG64(seed * 1000 + 5))
    out = []
    for k in np.asarray(key_map).tolist():
        key = keys[k]
        while True:
            r = 2 + rand_int(rng, key.bits + 64) % (key.n - 2)
            if math.gcd(r, key.n) == 1:
                break
        out.append(np.frombuffer(r.to_bytes(key.bits // 8, "big"), dtype=np.uint8))
    return np.concatenate(out) if out else np.zeros(0, np.uint8)


@dataclass
class ServingRequest:
    """One request of the serving workload: op 0 = encrypt, 1 = decrypt."""
    op: int
    msg_len: int
    keys: List[int]           # the request's key subset (indices into the table)
    key_map: np.ndarray       # chunk j under keys[j mod len(keys)]
    msg_seed: int             # seed of its message bytes (make_message)

    def message(self) -> np.ndarray:
        return make_message(self.msg_len, self.msg_seed)


def map_over_subset(msg_len: int, subset: Sequence[int], key_bits: Sequence[int]) -> np.ndarray:
    """Chunk j of a msg_len-byte message under subset[j mod len(subset)]."""
    out: List[int] = []
    off, j = 0, 0
    while off < msg_len:
        k = subset[j % len(subset)]
        out.append(k)
        off += key_bits[k] // 8 - 4
        j += 1
    return np.asarray(out, dtype=np.uint32)


def serving_requests(count: int, key_bits: Sequence[int], seed: int = 5, lo: int = 1024,
                     hi: int = 10 * 1024 * 1024, max_keys: int = 64, decrypt_share: float = 0.5
                     ) -> List[ServingRequest]:
    """Requests of the serving workload: sizes log-uniform in [lo, hi] bytes,
    1..max_keys distinct keys each (uniform count, drawn without replacement),
    encrypt or decrypt with probability 1 - decrypt_share / decrypt_share."""
    rng = np.random.Generator(np.random.PCG64(seed * 1000 + 4))
    reqs = []
    for i in range(count):
        size = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        k = int(rng.integers(1, max_keys + 1))
        subset = [int(x) for x in rng.choice(len(key_bits), size=min(k, len(key_bits)), replace=False)]
        op = int(rng.random() < decrypt_share)
        reqs.append(ServingRequest(op, size, subset, map_over_subset(size, subset, key_bits),
                                   seed * 100000 + i))
    return reqs


def poisson_arrivals(count: int, rate_per_s: float, seed: int = 5) -> np.ndarray:
    """Arrival offsets in seconds of a Poisson process of the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed * 1000 + 4 + 7919))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
