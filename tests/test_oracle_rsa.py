"""Pins for the oracle's RSA / PMKRSA layer (CPU only).

What fixes the expected values here, without the oracle's own code:
* Python's built-in ``pow`` (independent big-integer implementation);
* the RSA correctness identity decrypt(encrypt(m)) = m (Sec. 1.1) and the
  PMKRSA identity for the blinded form (Sec. 3.1);
* CRT decryption (Sec. 2.1) agreeing with plain c^d decryption;
* exhaustive bijection over Z_N for a 12-bit modulus;
* the classic p = 61, q = 53 example, whose numbers are checked by brute force
  (fixture in tests/golden/);
* closed forms of the chunk layout (chunk i of a round-robin map over equal key
  sizes starts at byte i*(kb-4)).
"""
import json
import math
import os
import random

import numpy as np
import pytest

import oracle
from paper_2111_11924_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_key(p, q, e=65537, use_lambda=True):
    return inputs.key_from_primes(p, q, e, use_lambda=use_lambda)


def test_textbook_key_3233_golden():
    with open(os.path.join(GOLDEN, "textbook_rsa_3233.json")) as f:
        g = json.load(f)
    p, q, e = g["p"], g["q"], g["e"]
    n = p * q
    # every stored number re-derived by brute-force search
    assert n == g["n"]
    lam = (p - 1) * (q - 1) // math.gcd(p - 1, q - 1)
    assert g["d_phi"] == next(d for d in range(1, (p - 1) * (q - 1)) if e * d % ((p - 1) * (q - 1)) == 1)
    assert g["d_lambda"] == next(d for d in range(1, lam) if e * d % lam == 1)
    assert g["qinv"] == next(x for x in range(1, p) if q * x % p == 1)
    c = 1
    for _ in range(e):
        c = c * g["m"] % n
    assert c == g["c"]
    # now the oracle, with both forms of d
    for d_key in ("d_phi", "d_lambda"):
        k = inputs.RsaKey(bits=12, n=n, e=e, d=g[d_key], p=p, q=q, dp=g[d_key] % (p - 1),
                          dq=g[d_key] % (q - 1), qinv=g["qinv"], n0inv=0, rr=0)
        T = oracle.KeyTable([k])
        assert oracle.rsa_int(T, 0, "enc", g["m"]) == g["c"]
        assert oracle.rsa_int(T, 0, "dec", g["c"]) == g["m"]
        assert oracle.rsa_int(T, 0, "crt", g["c"]) == g["m"]
    assert g["dp"] == g["d_phi"] % (p - 1) == g["d_lambda"] % (p - 1)
    assert g["dq"] == g["d_phi"] % (q - 1) == g["d_lambda"] % (q - 1)


def test_exhaustive_bijection_12bit():
    """Encryption permutes Z_N and CRT decryption inverts it, for every m."""
    k = small_key(61, 53, e=17)
    T = oracle.KeyTable([k])
    seen = set()
    for m in range(k.n):
        c = oracle.rsa_int(T, 0, "enc", m)
        assert c == pow(m, 17, k.n)
        seen.add(c)
        assert oracle.rsa_int(T, 0, "crt", c) == m
    assert len(seen) == k.n


@pytest.mark.parametrize("bits", [128, 256, 512, 1024])
def test_rsa_int_vs_pow_and_crt_equals_plain(bits):
    rng = random.Random(bits)
    key = inputs.make_key(bits, 777, 0)
    T = oracle.KeyTable([key])
    n = key.n
    specials = [0, 1, 2, n - 1, n - 2, key.p, key.q, key.p * 3, key.q * (key.p - 1)]
    randoms = [rng.randrange(n) for _ in range(6)]
    for m in specials + randoms:
        m %= n
        c = oracle.rsa_int(T, 0, "enc", m)
        assert c == pow(m, key.e, n)
        assert oracle.rsa_int(T, 0, "dec", c) == m
        assert oracle.rsa_int(T, 0, "crt", c) == m
    # fixed points of odd exponents
    for fp in (0, 1, n - 1):
        assert oracle.rsa_int(T, 0, "enc", fp) == fp


def test_d_phi_and_d_lambda_agree():
    key_l = inputs.make_key(256, 31, 3)
    key_f = inputs.key_from_primes(key_l.p, key_l.q, key_l.e, use_lambda=False)
    assert (key_l.dp, key_l.dq) == (key_f.dp, key_f.dq)
    Tl, Tf = oracle.KeyTable([key_l]), oracle.KeyTable([key_f])
    rng = random.Random(9)
    for _ in range(8):
        c = rng.randrange(key_l.n)
        assert oracle.rsa_int(Tl, 0, "dec", c) == oracle.rsa_int(Tf, 0, "dec", c)


def test_keygen_fields_are_consistent():
    import sympy

    for bits in (512, 1024, 2048):
        k = inputs.make_key(bits, 4242, 1)
        assert k.n.bit_length() == bits and k.p > k.q
        assert k.p.bit_length() == bits // 2 and k.q.bit_length() == bits // 2
        assert sympy.isprime(k.p) and sympy.isprime(k.q)
        lam = (k.p - 1) * (k.q - 1) // math.gcd(k.p - 1, k.q - 1)
        assert k.e * k.d % lam == 1
        assert k.dp == k.d % (k.p - 1) and k.dq == k.d % (k.q - 1)
        assert k.q * k.qinv % k.p == 1
        assert k.n * k.n0inv % (1 << 32) == (1 << 32) - 1
        assert k.rr == (1 << (2 * bits)) % k.n


def _msg_and_keys(cfg):
    w = inputs.config(cfg)
    return w, w.keys(), w.message(), w.key_map()


def test_config1_chunk_layout_closed_form():
    w, keys, msg, km = _msg_and_keys(1)
    T = oracle.KeyTable(keys)
    off, ln, cto, total = oracle.plan(T, km, len(msg))
    kb = 512 // 8
    n = len(km)
    assert n == -(-16384 // (kb - 4)) == 274
    assert (off == np.arange(n) * (kb - 4)).all()
    assert (ln[:-1] == kb - 4).all() and ln[-1] == 16384 - (n - 1) * (kb - 4) == 4
    assert (cto == np.arange(n) * kb).all() and total == n * kb
    assert (km == np.arange(n) % 8).all()


def test_config1_encrypt_vs_pow_and_roundtrip():
    w, keys, msg, km = _msg_and_keys(1)
    T = oracle.KeyTable(keys)
    ct = oracle.encrypt(T, msg, km)
    kb = 64
    for i in range(len(km)):
        k = keys[km[i]]
        chunk = bytes(msg[i * (kb - 4):(i + 1) * (kb - 4)])
        c = pow(int.from_bytes(chunk, "big"), k.e, k.n)
        assert bytes(ct[i * kb:(i + 1) * kb]) == c.to_bytes(kb, "big"), i
    pt, rc = oracle.decrypt(T, ct, len(msg), km, crt=True)
    assert rc == 0 and (pt == msg).all()
    pt2, rc2 = oracle.decrypt(T, ct, len(msg), km, crt=False)
    assert rc2 == 0 and (pt2 == msg).all()


def test_mixed_sizes_random_map_roundtrip():
    bits = [512, 1024, 512, 768, 1024]
    keys = inputs.make_keys(bits, 99)
    msg = inputs.make_message(5000, 99)
    km = inputs.random_map(len(msg), bits, 99)
    T = oracle.KeyTable(keys)
    off, ln, cto, total = oracle.plan(T, km, len(msg))
    caps = np.array([b // 8 - 4 for b in bits])
    assert ln.sum() == len(msg) and (ln[:-1] == caps[km[:-1]]).all()
    assert 1 <= ln[-1] <= caps[km[-1]]
    assert total == sum(bits[k] // 8 for k in km)
    ct = oracle.encrypt(T, msg, km)
    for i in range(len(km)):
        k = keys[km[i]]
        m = int.from_bytes(bytes(msg[off[i]:off[i] + ln[i]]), "big")
        assert int.from_bytes(bytes(ct[cto[i]:cto[i] + k.bits // 8]), "big") == pow(m, k.e, k.n)
    for crt in (True, False):
        pt, rc = oracle.decrypt(T, ct, len(msg), km, crt=crt)
        assert rc == 0 and (pt == msg).all()


def test_plan_rejects_wrong_chunk_counts():
    keys = inputs.make_keys([512, 512], 5)
    T = oracle.KeyTable(keys)
    km = inputs.round_robin_map(600, [512, 512])
    oracle.plan(T, km, 600)
    with pytest.raises(ValueError):
        oracle.plan(T, km[:-1], 600)
    with pytest.raises(ValueError):
        oracle.plan(T, np.concatenate([km, km[:1]]), 600)
    with pytest.raises(ValueError):
        oracle.plan(T, np.array([0, 7], dtype=np.uint32), 100)  # key index out of range
    off, ln, cto, total = oracle.plan(T, np.zeros(0, dtype=np.uint32), 0)
    assert total == 0 and len(off) == 0


def test_decrypt_flags_block_not_below_modulus():
    keys = inputs.make_keys([512], 6)
    T = oracle.KeyTable(keys)
    msg = inputs.make_message(120, 6)
    km = inputs.round_robin_map(120, [512])
    ct = oracle.encrypt(T, msg, km)
    bad = ct.copy()
    bad[0:64] = np.frombuffer(keys[0].n.to_bytes(64, "big"), dtype=np.uint8)  # c = N
    pt, rc = oracle.decrypt(T, bad, 120, km)
    assert rc == -3
    assert (pt[60:] == msg[60:]).all()  # the other chunks still decrypt


def test_blinded_pmkrsa_identity():
    """Sec. 3.1: c* = (r m)^e, c_R = r^e; decryption r' = c_R^d, m = (c*)^d r'^-1."""
    rng = random.Random(17)
    key = inputs.make_key(512, 12, 0)
    T = oracle.KeyTable([key])
    for _ in range(10):
        m = rng.randrange(key.n)
        while True:
            r = rng.randrange(1, key.n)
            if math.gcd(r, key.n) == 1:
                break
        cs, cr = oracle.blind_int(T, 0, "enc", m, r)
        assert cs == pow(r * m, key.e, key.n) == pow(m, key.e, key.n) * pow(r, key.e, key.n) % key.n
        assert cr == pow(r, key.e, key.n)
        m2, r2 = oracle.blind_int(T, 0, "dec", cs, cr)
        assert (m2, r2) == (m, r)
