"""Pins for the oracle's integer arithmetic (CPU only).

The oracle's schoolbook multiply, Knuth Algorithm D remainder and Algorithm 2
exponentiation are checked against Python's own big-integer arithmetic, an
independent implementation, on random and adversarial operands, and against
brute force and closed forms that do not depend on either implementation.
"""
import random

import pytest

import oracle

PATTERNS = [0, 1, 2, 0x7FFFFFFF, 0x80000000, 0x80000001, 0xFFFFFFFE, 0xFFFFFFFF]


def patterned(rng, nlimbs):
    x = 0
    for i in range(nlimbs):
        w = rng.choice(PATTERNS) if rng.random() < 0.6 else rng.getrandbits(32)
        x |= w << (32 * i)
    return x


def test_mul_matches_python_ints():
    rng = random.Random(101)
    for _ in range(3000):
        a = patterned(rng, rng.randint(1, 40)) if rng.random() < 0.5 else rng.getrandbits(rng.randint(1, 1300))
        b = patterned(rng, rng.randint(1, 40)) if rng.random() < 0.5 else rng.getrandbits(rng.randint(1, 1300))
        assert oracle.mul(a, b) == a * b


def test_mul_all_ones_carry_chain():
    for n in (1, 2, 16, 64, 128, 256):
        a = (1 << (32 * n)) - 1
        assert oracle.mul(a, a) == a * a
        assert oracle.mul(a, 1) == a
        assert oracle.mul(a, 0) == 0


def test_divmod_matches_python_ints():
    rng = random.Random(202)
    for _ in range(4000):
        vl = rng.randint(1, 34)
        ul = vl + rng.randint(0, 36)
        v = patterned(rng, vl) if rng.random() < 0.5 else rng.getrandbits(32 * vl)
        u = patterned(rng, ul) if rng.random() < 0.5 else rng.getrandbits(32 * ul)
        if v == 0:
            continue
        assert oracle.divmod_(u, v) == divmod(u, v), (hex(u), hex(v))


# Operands for which Algorithm D's quotient-digit estimate survives the
# second-limb test and is still one too large, so step D6 (add back) runs.
ADD_BACK_CASES = [
    (1 << 128, 0x10000000000000001),
    (1 << 128, 0x20000000000000001),
    (1 << 128, 0x800000000000000000000001),
    (1 << 128, 0x80000000000000007FFFFFFF),
    ((0x7FFFFFFF << 96) | (0x80000000 << 64), (0x80000000 << 64) | 1),
]


@pytest.mark.parametrize("u,v", ADD_BACK_CASES)
def test_divmod_add_back_step(u, v):
    assert oracle.divmod_(u, v) == divmod(u, v)


def test_divmod_small_and_degenerate():
    assert oracle.divmod_(0, 7) == (0, 0)
    assert oracle.divmod_(6, 7) == (0, 6)
    assert oracle.divmod_(7, 7) == (1, 0)
    assert oracle.divmod_((1 << 64) - 1, 0xFFFFFFFF) == divmod((1 << 64) - 1, 0xFFFFFFFF)
    with pytest.raises(ZeroDivisionError):
        oracle.divmod_(5, 0)


def test_modexp_matches_python_pow():
    rng = random.Random(303)
    for bits in (8, 31, 32, 33, 64, 100, 256, 512, 1024):
        for _ in range(12):
            m = rng.getrandbits(bits) | 1 | (1 << (bits - 1))
            x = rng.getrandbits(bits + 40)  # unreduced base too
            e = rng.getrandbits(rng.randint(1, bits))
            assert oracle.modexp(x, e, m) == pow(x, e, m)
    # even moduli are fine for the plain definition as well
    assert oracle.modexp(3, 1000, 1 << 40) == pow(3, 1000, 1 << 40)


def test_modexp_edge_exponents():
    m = (1 << 521) - 1
    assert oracle.modexp(12345, 0, m) == 1
    assert oracle.modexp(12345, 1, m) == 12345
    assert oracle.modexp(12345, 2, m) == 12345 ** 2 % m
    assert oracle.modexp(0, 5, m) == 0
    assert oracle.modexp(5, 7, 1) == 0  # everything is 0 mod 1


def test_modexp_brute_force_repeated_multiplication():
    """x^65537 mod N by 65,536 successive modular multiplications, for a 64-bit
    modulus built from two 32-bit primes."""
    p, q = 4294967291, 4294967279  # the two largest primes below 2^32
    n = p * q
    for x in (2, 3, 0xDEADBEEF12345, n - 2):
        y = x % n
        acc = y
        for _ in range(65536):
            acc = acc * y % n
        assert oracle.modexp(x, 65537, n) == acc


def test_fermat_little_theorem():
    for p in (65537, 4294967291, (1 << 127) - 1, (1 << 521) - 1):
        for a in (2, 3, 10 ** 9 + 7):
            assert oracle.modexp(a, p - 1, p) == 1
