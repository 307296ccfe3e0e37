"""GPU parity of the multi-prime CRT decryption (Sec. 2.1, multi-prime
variant): 3072-bit keys of 3 primes and 4096-bit keys of 4 primes.

The oracle is the plain definition m = C^d mod N (its c^d route, pinned in the
CPU suite); ciphertexts come from the oracle's encryption.  Every comparison is
exact (integer arithmetic).  Sizes span several 64-chunk tiles per key plus
ragged last tiles; edge blocks cover m = 0, 1, multiples of one and of two of
the primes (so C = 0 modulo those primes), and the largest chunk value.
"""
import numpy as np
import pytest

import oracle
from paper_2111_11924_amd import binding, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    c = binding.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def keys():
    return [inputs.make_mp_key(3072, 41, 0), inputs.make_mp_key(4096, 41, 1),
            inputs.make_mp_key(3072, 41, 2), inputs.make_mp_key(4096, 41, 3)]


def dev(torch, arr):
    a = np.ascontiguousarray(arr, dtype=np.uint8)
    t = torch.empty(max(len(a), 4), dtype=torch.uint8, device="cuda")
    if len(a):
        t[: len(a)].copy_(torch.from_numpy(a))
    return t


def gpu_decrypt(torch, ctx, keys, ct, km, msg_len):
    print(f"[gpu] multi-prime: {len(keys)} keys, {msg_len} bytes, {len(km)} chunks", flush=True)
    ctx.load_mp_keys(keys)
    d_ct = dev(torch, ct)
    d_msg = torch.zeros(max(msg_len, 4), dtype=torch.uint8, device="cuda")
    rc = binding.pmk_mp_decrypt(ctx.handle, d_ct, len(ct), km, d_msg, msg_len)
    torch.cuda.synchronize()
    return rc, d_msg[:msg_len].cpu().numpy()


def test_mp_tiles_and_ragged_tails(torch, ctx, keys):
    bits = [k.bits for k in keys]
    msg_len = 150 * 380 + 90 * 508 + 77 * 380 + 3 * 508 + 11
    km = inputs.round_robin_map(msg_len, bits)
    msg = inputs.make_message(msg_len, 42)
    T = oracle.KeyTable(keys)
    ct = oracle.encrypt(T, msg, km)
    rc, pt = gpu_decrypt(torch, ctx, keys, ct, km, msg_len)
    assert rc == binding.PMK_OK, binding.pmk_last_error(ctx.handle)
    bad = np.nonzero(pt != msg)[0]
    assert len(bad) == 0, f"plaintext differs at byte {bad[0]} ({len(bad)} bytes)"


@pytest.mark.parametrize("which", [0, 1])
def test_mp_edge_blocks_against_oracle(torch, ctx, keys, which):
    k = keys[which]
    kb = k.bits // 8
    cap = kb - 4
    vals = [0, 1, 2, k.primes[0], k.primes[-1] * 3, k.primes[0] * k.primes[1], (1 << (8 * cap)) - 1,
            k.primes[1] - 1]
    msg = np.concatenate([np.frombuffer(v.to_bytes(cap, "big"), dtype=np.uint8) for v in vals])
    km = np.zeros(len(vals), dtype=np.uint32)
    T = oracle.KeyTable([k])
    ct = oracle.encrypt(T, msg, km)
    ref, rc_ref = oracle.decrypt(T, ct, len(msg), km, crt=False)
    assert rc_ref == 0 and (ref == msg).all()
    rc, pt = gpu_decrypt(torch, ctx, [k], ct, km, len(msg))
    assert rc == binding.PMK_OK, binding.pmk_last_error(ctx.handle)
    assert (pt == ref).all()


def test_mp_range_error_and_size_checks(torch, ctx, keys):
    k = keys[0]
    kb = k.bits // 8
    ctx.load_mp_keys([k])
    km = np.zeros(2, dtype=np.uint32)
    msg_len = 2 * (kb - 4)
    ct = np.zeros(2 * kb, dtype=np.uint8)
    ct[kb:] = np.frombuffer(k.n.to_bytes(kb, "big"), dtype=np.uint8)  # second block C = N
    d_ct = dev(torch, ct)
    d_msg = torch.zeros(msg_len, dtype=torch.uint8, device="cuda")
    assert binding.pmk_mp_decrypt(ctx.handle, d_ct, len(ct), km, d_msg, msg_len) == binding.PMK_ERANGE
    assert binding.pmk_mp_decrypt(ctx.handle, d_ct, len(ct) - 1, km, d_msg, msg_len) == binding.PMK_ESIZE
    assert binding.pmk_mp_decrypt(ctx.handle, d_ct, len(ct), np.array([0, 1], dtype=np.uint32), d_msg,
                                  msg_len) == binding.PMK_EKEY
    # empty message: nothing to do
    assert binding.pmk_mp_decrypt(ctx.handle, d_ct, 0, np.zeros(0, dtype=np.uint32), d_msg, 0) == binding.PMK_OK
    # a valid call after the errors still decrypts
    ct_ok = np.zeros(2 * kb, dtype=np.uint8)
    ct_ok[kb - 1] = 1  # C = 1 -> m = 1
    rc, pt = gpu_decrypt(torch, ctx, [k], ct_ok, km, msg_len)
    assert rc == binding.PMK_OK
    want = np.zeros(msg_len, dtype=np.uint8)
    want[kb - 5] = 1
    assert (pt == want).all()
