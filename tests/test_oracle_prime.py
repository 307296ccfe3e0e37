"""Pins of the oracle's primality routines (key generation): values fixed by
number theory, not by the routines themselves."""
import oracle

# strong pseudoprimes to base 2 (odd composites that pass Miller-Rabin with a = 2)
STRONG_PSP_BASE2 = [2047, 3277, 4033, 4681, 8321, 15841, 29341, 42799, 49141, 52633]


def test_small_primes_sieve():
    p = oracle.small_odd_primes(4096)
    assert len(p) == 563 and p[:5] == [3, 5, 7, 11, 13] and p[-1] == 4093
    # brute force
    assert p == [n for n in range(3, 4096, 2) if all(n % k for k in range(3, int(n ** 0.5) + 1, 2))]


def test_strong_pseudoprimes_pass_base_2_only():
    for m in STRONG_PSP_BASE2:
        assert oracle.miller_rabin(m, [2]), m            # the definition of a strong pseudoprime
        assert not all(m % k for k in range(2, int(m ** 0.5) + 1)), m  # and they are composite
    assert not oracle.miller_rabin(2047, [3])            # base 3 witnesses 2047 = 23 * 89


def test_carmichael_numbers_are_caught():
    # Carmichael numbers fool Fermat's test for every coprime base, not Miller-Rabin
    for m in (561, 1105, 1729, 2465, 2821, 6601, 8911):
        assert pow(2, m - 1, m) == 1
        assert not oracle.miller_rabin(m, [2, 3, 5, 7])


def test_primes_pass_every_base():
    for m in ((1 << 61) - 1, (1 << 89) - 1, (1 << 127) - 1, (1 << 521) - 1):  # Mersenne primes
        assert oracle.miller_rabin(m, [2, 3, 5, 7, 11, 13, 17, m - 2])


def test_products_of_primes_are_composite():
    p, q = (1 << 61) - 1, (1 << 89) - 1
    assert not oracle.miller_rabin(p * q, [2])
    assert not oracle.trial_division_pass(3 * 4093 * p)
    assert oracle.trial_division_pass(p * q)
