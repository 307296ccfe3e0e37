"""GPU test of the allocation-free decryption entry point (pmk_decrypt_noalloc)
through the C ABI: byte-identical to pmk_decrypt, on two calls in a row (the
second with a smaller input and an out-of-range block, so stale scratch
contents from the first would show), and its size limit."""
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


def dev(torch, arr):
    a = np.ascontiguousarray(arr, dtype=np.uint8)
    t = torch.empty(max(len(a), 4), dtype=torch.uint8, device="cuda")
    if len(a):
        t[: len(a)].copy_(torch.from_numpy(a))
    return t


def both(torch, ctx, ct, km, msg_len):
    """(status, bytes) of pmk_decrypt and of pmk_decrypt_noalloc on the same input."""
    outs = []
    for fn in (binding.pmk_decrypt, binding.pmk_decrypt_noalloc):
        d_ct = dev(torch, ct)
        d_pt = torch.full((max(msg_len, 4),), 0x5A, dtype=torch.uint8, device="cuda")
        rc = fn(ctx.handle, d_ct, len(ct), km, d_pt, msg_len)
        torch.cuda.synchronize()
        outs.append((rc, d_pt[:msg_len].cpu().numpy()))
    return outs


def test_noalloc_matches_pmk_decrypt_twice(torch):
    bits = [1024, 2048, 4096, 512, 3072]
    keys = inputs.make_keys(bits, 970)
    T = oracle.KeyTable(keys)
    ctx = binding.Context(0)
    try:
        ctx.load_keys(keys)
        # call 1: about 2 MB over every class
        msg1 = inputs.make_message(2_000_000 + 5, 970)
        km1 = inputs.random_map(len(msg1), bits, 970)
        ct1 = oracle.encrypt(T, msg1, km1)
        print(f"[gpu] noalloc call 1: {len(km1)} chunks", flush=True)
        (rc_a, pt_a), (rc_b, pt_b) = both(torch, ctx, ct1, km1, len(msg1))
        assert rc_a == rc_b == binding.PMK_OK
        assert (pt_b == pt_a).all() and (pt_b == msg1).all()
        # call 2: smaller, two classes only, one block equal to N
        sub = [0, 1]
        msg2 = inputs.make_message(300_000 + 1, 971)
        km2 = inputs.map_over_subset(len(msg2), sub, bits)
        ct2 = oracle.encrypt(T, msg2, km2)
        kb = keys[int(km2[3])].bits // 8
        off = sum(keys[int(k)].bits // 8 for k in km2[:3])
        ct2[off:off + kb] = np.frombuffer(keys[int(km2[3])].n.to_bytes(kb, "big"), np.uint8)
        print(f"[gpu] noalloc call 2: {len(km2)} chunks", flush=True)
        (rc_a, pt_a), (rc_b, pt_b) = both(torch, ctx, ct2, km2, len(msg2))
        ref, rc_o = oracle.decrypt(T, ct2, len(msg2), km2)
        assert rc_o == -3 and rc_a == rc_b == binding.PMK_ERANGE
        assert (pt_b == pt_a).all() and (pt_b == ref).all()
        # empty message
        assert binding.pmk_decrypt_noalloc(ctx.handle, None, 0, np.zeros(0, np.uint32), None, 0) == binding.PMK_OK
    finally:
        ctx.close()


def test_noalloc_refuses_beyond_its_limit(torch):
    keys = inputs.make_keys([128], 972)
    ctx = binding.Context(0)
    try:
        ctx.load_keys(keys)
        n = 65_537  # one chunk over the limit (12-byte chunks)
        msg_len = n * 12
        km = np.zeros(n, np.uint32)
        d_ct = torch.zeros(n * 16, dtype=torch.uint8, device="cuda")
        d_pt = torch.zeros(msg_len, dtype=torch.uint8, device="cuda")
        rc = binding.pmk_decrypt_noalloc(ctx.handle, d_ct, n * 16, km, d_pt, msg_len)
        assert rc == binding.PMK_ESIZE
        assert "at most 65536" in binding.pmk_last_error(ctx.handle)
        # at the limit it runs (zero blocks decrypt to zero chunks)
        n = 65_536
        rc = binding.pmk_decrypt_noalloc(ctx.handle, d_ct, n * 16, km[:n], d_pt, n * 12)
        torch.cuda.synchronize()
        assert rc == binding.PMK_OK
        assert not d_pt[: n * 12].any().item()
    finally:
        ctx.close()
