"""Pins of the oracle at the sizes the GPU is checked against (CPU only).

Every expected value here comes from outside the oracle:
* Python's built-in integers (``pow``, ``divmod``, ``*``), an independent
  big-integer implementation, for textbook RSA c = m^e mod N and m = c^d mod N
  (Sec. 1.1) at 2048-8192-bit moduli;
* the defining congruences of CRT decryption (Sec. 2.1): the result r is the
  unique value below N with r = c^dp mod p and r = c^dq mod q, checked with
  ``pow`` modulo each prime, for CRT exponents of any shape;
* the defining identity of blinded decryption (Sec. 3.1, Eqs. 3-10):
  m (c_R^d) = (c*)^d mod N;
* the multi-prime variant of Sec. 2.1, whose oracle is the plain c^d route;
* the RSA correctness identity decrypt(encrypt(m)) = m over every chunk of the
  1 MiB workload and over >= 4,096 sampled chunks per modulus size of the mixed
  25 MiB and the 100 MiB workloads, with every ciphertext block also equal to
  ``pow``.

The keys are the seeded inputs stored in tests/golden/large_keys.json
(written by tests/golden/make_large_keys.py from the package's key generator),
rechecked here before use.
"""
import json
import math
import os
import random
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2111_11924_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SIZES = (2048, 3072, 4096, 6144, 8192)
# PMK_PIN_FULL=1: decrypt every sampled chunk of the large workloads (about
# 4,096 per modulus size, several minutes); by default a smaller per-size
# sample is decrypted while every sampled chunk's encryption is still checked.
FULL = os.environ.get("PMK_PIN_FULL", "") == "1"


def pmap(fn, items):
    """fn over items on all host cores (the oracle's ctypes calls release the
    interpreter lock), results in order."""
    items = list(items)
    with ThreadPoolExecutor(max_workers=os.cpu_count() or 1) as ex:
        return list(ex.map(fn, items))


@pytest.fixture(scope="module")
def large_keys():
    with open(os.path.join(GOLDEN, "large_keys.json")) as f:
        obj = json.load(f)
    keys = {k["bits"]: inputs.RsaKey.from_json(k) for k in obj["keys"]}
    assert sorted(keys) == list(SIZES)
    return keys


def test_large_keys_are_valid_rsa_keys(large_keys):
    import sympy

    for bits, k in large_keys.items():
        assert k.n == k.p * k.q and k.n.bit_length() == bits and k.p > k.q
        assert sympy.isprime(k.p) and sympy.isprime(k.q), bits
        lam = (k.p - 1) * (k.q - 1) // math.gcd(k.p - 1, k.q - 1)
        assert k.e * k.d % lam == 1
        assert (k.dp, k.dq) == (k.d % (k.p - 1), k.d % (k.q - 1))
        assert k.q * k.qinv % k.p == 1


# ---------------------------------------------------------------- Algorithm D at size

def _limbs_random(rng, n, patterned):
    if not patterned:
        return rng.getrandbits(32 * n) | (1 << (32 * n - 1)) * rng.getrandbits(1)
    pats = [0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF]
    x = 0
    for i in range(n):
        x |= (rng.choice(pats) if rng.random() < 0.7 else rng.getrandbits(32)) << (32 * i)
    return x


def test_divmod_large_operands():
    """Dividends of 128-520 limbs by divisors of 64-256 limbs (the sizes of the
    reductions of 2048-8192-bit products), random and limb-patterned."""
    rng = random.Random(5150)
    for it in range(400):
        vl = rng.randint(64, 256)
        ul = rng.randint(max(128, vl), 520)
        v = _limbs_random(rng, vl, it % 2 == 1)
        u = _limbs_random(rng, ul, it % 3 == 1)
        if v == 0:
            continue
        assert oracle.divmod_(u, v) == divmod(u, v), (it, ul, vl)


def _step_adds_back(u, v, j):
    """Whether quotient step j of Knuth's Algorithm D on (u, v) -- divisor with
    its top bit set (no normalising shift), every earlier step having taken a
    zero digit so the dividend limbs are still u's -- keeps an estimate that is
    one too large, so that the add-back step (D6) runs."""
    B = 1 << 32
    n = (v.bit_length() + 31) // 32
    limb = lambda x, i: (x >> (32 * i)) & (B - 1)
    top = limb(u, j + n) * B + limb(u, j + n - 1)
    qhat, rhat = divmod(top, limb(v, n - 1))
    while qhat >= B or qhat * limb(v, n - 2) > rhat * B + limb(u, j + n - 2):
        qhat -= 1
        rhat += limb(v, n - 1)
        if rhat >= B:
            break
    window = (u >> (32 * j)) % B ** (n + 1)
    return qhat * v > window


@pytest.mark.parametrize("n", [64, 128, 256])
def test_divmod_add_back_at_size(n):
    """Operands built so that the quotient estimate from the top two divisor
    limbs survives the second-limb test and is still one too large: the top
    three dividend limbs equal q0 times the top two divisor limbs, the divisor's
    lower limbs are all ones, so the full product q0 v exceeds the dividend by
    q0 (B^(n-2) - 1).  Lower dividend limbs below the first step are random."""
    rng = random.Random(n)
    B = 1 << 32
    for _ in range(20):
        vt = (rng.getrandbits(31) | (1 << 31)) * B + rng.getrandbits(32)  # top two limbs, top bit set
        v = vt * B ** (n - 2) + (B ** (n - 2) - 1)
        q0 = rng.randrange(1, B)
        k = rng.randint(0, 200)  # further quotient limbs after the first
        u = (q0 * vt) * B ** (n - 2 + k) + rng.getrandbits(32 * k)
        # the top limb of u stays below the divisor's, so the step above takes a
        # zero digit and step k meets the constructed limbs
        if (u >> (32 * (n + k))) >= (v >> (32 * (n - 1))):
            continue
        assert _step_adds_back(u, v, k)
        assert oracle.divmod_(u, v) == divmod(u, v)


def test_limb_capacity_is_refused_not_truncated():
    big = (1 << (32 * 520)) - 1
    assert oracle.divmod_(big, 12345) == divmod(big, 12345)
    with pytest.raises(OverflowError):
        oracle.divmod_(1 << (32 * 520), 12345)  # 521 limbs
    with pytest.raises(OverflowError):
        oracle.mul(1 << (32 * 300), 1 << (32 * 230))
    assert oracle.mul((1 << (32 * 260)) - 1, (1 << (32 * 260)) - 1) == ((1 << (32 * 260)) - 1) ** 2
    with pytest.raises(OverflowError):
        oracle.modexp(3, 5, (1 << (32 * 260)) + 1)  # modulus of 261 limbs
    m = (1 << (32 * 260)) - 3
    assert oracle.modexp(3, 7, m) == pow(3, 7, m)


# ---------------------------------------------------------------- RSA at 2048-8192 bits

def _specials(k):
    n = k.n
    return [0, 1, 2, n - 1, n - 2, k.p, k.q, 3 * k.p, k.q * (k.p - 1), (1 << (k.bits - 32)) - 1]


@pytest.mark.parametrize("bits", SIZES)
def test_rsa_int_large_vs_pow(large_keys, bits):
    k = large_keys[bits]
    T = oracle.KeyTable([k])
    rng = random.Random(bits + 1)
    values = _specials(k) + [rng.randrange(k.n) for _ in range(4)]
    cts = pmap(lambda m: oracle.rsa_int(T, 0, "enc", m), values)
    for m, c in zip(values, cts):
        assert c == pow(m, k.e, k.n), (bits, m)
    assert pmap(lambda c: oracle.rsa_int(T, 0, "crt", c), cts) == values
    # plain c^d route and CRT route on ciphertexts not made by the oracle
    cs = [rng.randrange(k.n), k.n - 1, k.p]
    refs = [pow(c, k.d, k.n) for c in cs]
    jobs = [(mode, c) for c in cs for mode in ("dec", "crt")]
    got = pmap(lambda j: oracle.rsa_int(T, 0, j[0], j[1]), jobs)
    assert got == [r for r in refs for _ in range(2)]


def _shaped_crt_exponents(h):
    return [
        (0, 1),
        (1, 3),
        (1 << (h - 2), (1 << (h - 2)) | 1),
        ((1 << (h - 2)) | 1, (1 << 200) | (1 << 130) | 5),
        ((0b101101 << (h - 8)) | (1 << 65) | 1, (1 << 63) | (1 << 64)),
        ((1 << (h - 3)) - 1, 7 << 70),
    ]


@pytest.mark.parametrize("bits", SIZES)
def test_crt_route_with_shaped_exponents(large_keys, bits):
    """CRT decryption with CRT exponents of any shape (zero, one, single bits,
    zero runs longer than 64 bits) is the unique r < N with r = c^dp mod p and
    r = c^dq mod q."""
    base = large_keys[bits]
    rng = random.Random(bits + 2)
    jobs = []
    for dp, dq in _shaped_crt_exponents(bits // 2):
        f = dict(base.__dict__)
        f.update(dp=dp % base.p, dq=dq % base.q)
        T = oracle.KeyTable([inputs.RsaKey(**f)])
        for c in (rng.randrange(base.n), rng.randrange(1 << (bits - 8)), base.q * 5):
            jobs.append((T, f["dp"], f["dq"], c))
    got = pmap(lambda j: oracle.rsa_int(j[0], 0, "crt", j[3]), jobs)
    for (_, dp, dq, c), r in zip(jobs, got):
        assert r < base.n
        assert r % base.p == pow(c % base.p, dp, base.p)
        assert r % base.q == pow(c % base.q, dq, base.q)


@pytest.mark.parametrize("bits", SIZES)
def test_blind_int_large(large_keys, bits):
    """Sec. 3.1: c* = (r m)^e, c_R = r^e; decryption gives back (m, r)."""
    k = large_keys[bits]
    T = oracle.KeyTable([k])
    rng = random.Random(bits + 3)
    pairs = [(rng.randrange(k.n), rng.randrange(2, k.n)) for _ in range(4)]
    assert all(math.gcd(r, k.n) == 1 for _, r in pairs)
    enc = pmap(lambda mr: oracle.blind_int(T, 0, "enc", mr[0], mr[1]), pairs)
    for (m, r), (cs, cr) in zip(pairs, enc):
        assert cs == pow(r * m % k.n, k.e, k.n)
        assert cr == pow(r, k.e, k.n)
    assert pmap(lambda c: oracle.blind_int(T, 0, "dec", c[0], c[1]), enc) == pairs


@pytest.mark.parametrize("bits", SIZES)
def test_blind_int_with_short_private_exponents(large_keys, bits):
    """Blinded decryption with private exponents of unusual shape (the inputs
    of the GPU's blinded parity test): the result m satisfies
    m (c_R^d) = (c*)^d mod N, and r' = c_R^d."""
    base = large_keys[bits]
    h = bits // 2
    rng = random.Random(bits + 4)
    jobs = []
    for d in (1, 3, (1 << 70) + 5, (1 << (h - 3)) - 1, (1 << (h - 2)) | 1, (1 << 100) | (1 << 37)):
        f = dict(base.__dict__)
        f.update(d=d, dp=d, dq=d)
        cs, cr = rng.randrange(1 << (bits - 8)), rng.randrange(1 << (bits - 8))
        assert math.gcd(cr, base.n) == 1
        jobs.append((oracle.KeyTable([inputs.RsaKey(**f)]), d, cs, cr))
    got = pmap(lambda j: oracle.blind_int(j[0], 0, "dec", j[2], j[3]), jobs)
    for (_, d, cs, cr), (m, r1) in zip(jobs, got):
        assert m < base.n
        assert r1 == pow(cr, d, base.n)
        assert m * r1 % base.n == pow(cs, d, base.n)


# ---------------------------------------------------------------- multi-prime (Sec. 2.1)

@pytest.mark.parametrize("bits", [3072, 4096])
def test_multi_prime_cd_route(bits):
    """The oracle of multi-prime decryption is the plain route m = C^d mod N
    (N the product of bits/1024 primes)."""
    k = inputs.make_mp_key(bits, 41, 0 if bits == 3072 else 1)
    assert math.prod(k.primes) == k.n and len(k.primes) == bits // 1024
    T = oracle.KeyTable([k])
    rng = random.Random(bits + 5)
    cs = [rng.randrange(k.n), k.primes[0] * 7, k.primes[0] * k.primes[1], k.n - 1, 0, 1]
    assert pmap(lambda c: oracle.rsa_int(T, 0, "dec", c), cs) == [pow(c, k.d, k.n) for c in cs]
    for m in (rng.randrange(k.n), (1 << (bits - 32)) - 1):
        c = oracle.rsa_int(T, 0, "enc", m)
        assert c == pow(m, k.e, k.n)
        assert oracle.rsa_int(T, 0, "dec", c) == m
    # whole-message plain route over several chunks
    msg = inputs.make_message(3 * (bits // 8 - 4) + 17, bits)
    km = np.zeros(4, np.uint32)
    ct = oracle.encrypt(T, msg, km)
    pt, rc = oracle.decrypt(T, ct, len(msg), km, crt=False)
    assert rc == 0 and (pt == msg).all()


# ---------------------------------------------------------------- whole workloads

def _chunk_layout(key_bits, km, msg_len):
    """Offsets and lengths of every chunk (chunk i: kb - 4 bytes of its key,
    the last one the remainder), computed here independently of the oracle."""
    caps = np.array([b // 8 - 4 for b in key_bits], dtype=np.int64)[km]
    ln = caps.copy()
    off = np.concatenate([[0], np.cumsum(caps)[:-1]])
    ln[-1] = msg_len - off[-1]
    assert 1 <= ln[-1] <= caps[-1]
    return off, ln


def _pin_sample(keys, msg, km, idx, dec_pos=None):
    """Encrypt the chunks idx (a sub-message of exactly those chunks) with the
    oracle: every block must equal pow(m, e, N).  CRT decryption of the blocks
    at positions dec_pos of idx (all of them by default) and plain decryption of
    the first few must give the chunks back."""
    key_bits = [k.bits for k in keys]
    off, ln = _chunk_layout(key_bits, km, len(msg))
    sub_km = km[idx]
    parts = [msg[off[i]:off[i] + ln[i]] for i in idx.tolist()]
    # a chunk shorter than its key's capacity can only be the last one
    assert all(len(p) == key_bits[k] // 8 - 4 for p, k in zip(parts[:-1], sub_km[:-1].tolist()))
    sub = np.concatenate(parts).astype(np.uint8)
    T = oracle.KeyTable(keys)
    ct = oracle.encrypt(T, sub, sub_km)
    blocks, pos = [], 0
    for p, k in zip(parts, sub_km.tolist()):
        kb = key_bits[k] // 8
        c = pow(int.from_bytes(bytes(p), "big"), keys[k].e, keys[k].n)
        assert bytes(ct[pos:pos + kb]) == c.to_bytes(kb, "big")
        blocks.append(ct[pos:pos + kb])
        pos += kb
    assert pos == len(ct)

    def roundtrip(pos_list, crt):
        pos_list = list(pos_list)
        dk = sub_km[pos_list]
        dm = np.concatenate([parts[j] for j in pos_list]).astype(np.uint8)
        dc = np.concatenate([blocks[j] for j in pos_list]).astype(np.uint8)
        pt, rc = oracle.decrypt(T, dc, len(dm), dk, crt=crt)
        assert rc == 0 and (pt == dm).all()

    roundtrip(range(len(idx)) if dec_pos is None else dec_pos, True)
    roundtrip(range(min(len(idx), 16)), False)


def test_config2_every_chunk_vs_pow():
    """The 1 MiB workload (64 x 2048-bit keys, 4,162 chunks) in full."""
    w = inputs.config(2)
    keys, msg, km = w.keys(), w.message(), w.key_map()
    assert len(km) == 4162
    _pin_sample(keys, msg, km, np.arange(len(km)))


def _per_class_sample(keys, km, per_class, seed):
    rng = np.random.default_rng(seed)
    bits = np.array([k.bits for k in keys])[km]
    picks = [np.array([len(km) - 1])]  # the ragged last chunk
    for b in sorted(set(bits.tolist())):
        rows = np.nonzero(bits == b)[0]
        rows = rows[rows != len(km) - 1]
        picks.append(rows if len(rows) <= per_class else rng.choice(rows, per_class, replace=False))
    return np.unique(np.concatenate(picks))


def _decrypt_positions(keys, km, idx, seed):
    """Positions within idx whose CRT decryption is checked: all of them with
    PMK_PIN_FULL=1, else 1,024 per modulus size up to 2048 bits and 256 above
    (the oracle's CRT decryption of a 4096-bit block takes about 0.2 s of one
    core), always including the last one."""
    if FULL:
        return None
    rng = np.random.default_rng(seed)
    bits = np.array([k.bits for k in keys])[km[idx]]
    out = [np.array([len(idx) - 1])]
    for b in sorted(set(bits.tolist())):
        rows = np.nonzero(bits == b)[0]
        want = 1024 if b <= 2048 else 256
        out.append(rows if len(rows) <= want else rng.choice(rows, want, replace=False))
    return np.unique(np.concatenate(out))


@pytest.mark.slow
def test_config3_sampled_chunks_per_size_vs_pow():
    """The mixed 25 MiB workload: 4,096 sampled chunks of each modulus size,
    every one encrypted and checked against pow."""
    w = inputs.config(3)
    keys, msg, km = w.keys(), w.message(), w.key_map()
    idx = _per_class_sample(keys, km, 4096, 3)
    sizes = np.array([k.bits for k in keys])[km[idx]]
    assert all((sizes == b).sum() >= 4096 for b in (1024, 2048, 3072, 4096))
    _pin_sample(keys, msg, km, idx, _decrypt_positions(keys, km, idx, 33))


@pytest.mark.slow
def test_config4_sampled_chunks_vs_pow():
    """The 100 MiB workload (416,102 chunks under 256 2048-bit keys): 4,096
    sampled chunks plus the ragged last one."""
    w = inputs.config(4)
    keys, msg, km = w.keys(), w.message(), w.key_map()
    idx = _per_class_sample(keys, km, 4096, 4)
    _pin_sample(keys, msg, km, idx, _decrypt_positions(keys, km, idx, 44))
