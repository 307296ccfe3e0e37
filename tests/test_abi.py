"""Host-side tests of the C ABI (no GPU): the library loads, exports every
function include/pmk.h declares, validates keys and chunk plans.

The plan checks are compared with the oracle's own chunk planning, which is an
independent implementation of the same layout rules."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2111_11924_amd import binding, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "pmk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pmk_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = binding.load_library()
    names = header_functions()
    assert "pmk_keys_load" in names and "pmk_decrypt_plan" in names
    for name in names:
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr)


def test_binding_covers_the_abi():
    for name in header_functions():
        assert callable(getattr(binding, name)), name


@pytest.mark.parametrize("bits", [128, 256, 512, 1024, 2048])
def test_key_check_accepts_generated_keys(bits):
    k = inputs.make_key(bits, 55, 0)
    assert binding.pmk_key_check(k) == (binding.PMK_OK, "")


def _mut(k, **kw):
    d = dict(k.__dict__)
    d.update(kw)
    return inputs.RsaKey(**d)


def test_key_check_rejects_bad_material():
    k = inputs.make_key(512, 56, 0)
    bad = {
        "n0inv": _mut(k, n0inv=(k.n0inv + 1) % (1 << 32)),
        "rr": _mut(k, rr=(k.rr + 1) % k.n),
        "p*q": _mut(k, n=k.n + 2, rr=pow(2, 1024, k.n + 2), n0inv=(-pow(k.n + 2, -1, 1 << 32)) % (1 << 32)),
        "qinv": _mut(k, qinv=(k.qinv + 1) % k.p),
        "p<q": _mut(k, p=k.q, q=k.p),
        "even e": _mut(k, e=65536),
        "dp>=p": _mut(k, dp=k.p),
    }
    for what, key in bad.items():
        rc, msg = binding.pmk_key_check(key)
        assert rc == binding.PMK_EINVAL, (what, rc, msg)
        assert msg, what


def test_key_check_rejects_sizes():
    k = inputs.make_key(512, 57, 0)
    rc, _ = binding.pmk_key_check(_mut(k, bits=520))
    assert rc == binding.PMK_EINVAL


def test_plan_validate_matches_oracle_plan():
    bits = [512, 1024, 2048, 768]
    keys = inputs.make_keys(bits, 58)
    T = oracle.KeyTable(keys)
    for msg_len in (1, 59, 60, 61, 1000, 4096, 12345):
        km = inputs.random_map(msg_len, bits, msg_len)
        rc, ct_len = binding.pmk_plan_validate(bits, km, msg_len)
        assert rc == binding.PMK_OK
        assert ct_len == oracle.plan(T, km, msg_len)[3]


def test_plan_validate_errors():
    bits = [512, 512]
    km = inputs.round_robin_map(600, bits)
    assert binding.pmk_plan_validate(bits, km, 600)[0] == binding.PMK_OK
    assert binding.pmk_plan_validate(bits, km[:-1], 600)[0] == binding.PMK_ESIZE
    assert binding.pmk_plan_validate(bits, np.concatenate([km, km[:1]]), 600)[0] == binding.PMK_ESIZE
    bad = km.copy()
    bad[3] = 2
    assert binding.pmk_plan_validate(bits, bad, 600)[0] == binding.PMK_EKEY
    assert binding.pmk_plan_validate(bits, np.zeros(0, np.uint32), 0) == (binding.PMK_OK, 0)
    assert binding.pmk_plan_validate(bits, np.zeros(1, np.uint32), 0)[0] == binding.PMK_ESIZE
    assert binding.pmk_plan_validate([500], [0], 10)[0] == binding.PMK_EINVAL


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError):
        binding.load_library(str(tmp_path / "libpmk.so"))


# ---------- multi-prime keys (host-side checks) -----------------------------------------

@pytest.fixture(scope="module")
def mp_keys():
    return [inputs.make_mp_key(3072, 57, 0), inputs.make_mp_key(4096, 57, 1)]


def test_mp_keys_satisfy_the_rsa_identity(mp_keys):
    """Generated multi-prime keys: N = product of the primes, e d = 1 modulo
    every p_i - 1, so (m^e)^d = m mod N (Sec. 1.1 correctness)."""
    for k in mp_keys:
        n = 1
        for p, d in zip(k.primes, k.exps):
            n *= p
            assert p.bit_length() == 1024 and (k.e * d) % (p - 1) == 1
        assert n == k.n and n.bit_length() == k.bits
        m = 0x1234567 ** 40 % k.n
        assert pow(pow(m, k.e, k.n), k.d, k.n) == m


def test_mp_key_check_accepts_generated_keys(mp_keys):
    for k in mp_keys:
        assert binding.pmk_mp_key_check(k) == (binding.PMK_OK, "")


def _mp_mut(k, **kw):
    d = dict(k.__dict__)
    d.update(kw)
    return inputs.MpKey(**d)


def test_mp_key_check_rejects_bad_material(mp_keys):
    k = mp_keys[0]
    p0, p1, p2 = k.primes
    small = (1 << 1023) - 1  # odd, 1023 bits
    bad = {
        "bits": _mp_mut(k, bits=5120),
        "bits vs nprimes": _mp_mut(k, bits=4096),
        "nprimes": _mp_mut(k, primes=[p0, p1], exps=k.exps[:2]),
        "product": _mp_mut(k, n=k.n + 2),
        "prime size": _mp_mut(k, primes=[small, p1, p2], n=small * p1 * p2 | (1 << 3071)),
        "repeated prime": _mp_mut(k, primes=[p0, p0, p2], n=p0 * p0 * p2),
        "d_i >= p_i": _mp_mut(k, exps=[p0, k.exps[1], k.exps[2]]),
        "even n": _mp_mut(k, n=k.n - 1),
    }
    for what, key in bad.items():
        rc, msg = binding.pmk_mp_key_check(key)
        assert rc == binding.PMK_EINVAL, what
        assert msg, what
