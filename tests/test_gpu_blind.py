"""GPU parity of blinded PMKRSA (Sec. 3.1, Algorithm 1): c* = (r m)^e, c_R = r^e
per chunk, and m = (c*)^d (c_R^d)^-1 mod N, each compared exactly with the
oracle's per-chunk blinding routine and by round trip over whole messages."""
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


def dev(torch, arr):
    a = np.ascontiguousarray(arr, dtype=np.uint8)
    t = torch.empty(max(len(a), 4), dtype=torch.uint8, device="cuda")
    if len(a):
        t[: len(a)].copy_(torch.from_numpy(a))
    return t


def chunk_spans(keys, km, msg_len):
    """(msg_off, len, ct_off, kb) per chunk."""
    out, off, ct = [], 0, 0
    for k in km.tolist():
        kb = keys[k].bits // 8
        ln = min(kb - 4, msg_len - off)
        out.append((off, ln, ct, kb))
        off += ln
        ct += kb
    return out


@pytest.mark.parametrize("bits,nbytes,samples", [
    ([512, 1024, 256], 64 * 3 * 60 + 11, 24),   # several tiles per class, ragged
    ([128, 192], 64 * 3 * 12 + 5, 24),          # the two smallest classes (192 bits runs in the 256-bit one)
    ([2048, 2048], 140 * 252 + 5, 12),
    ([3072, 4096, 1536], 40 * 400 + 3, 6),      # lane-group classes and a non-class size
])
def test_blinded_encrypt_decrypt_match_oracle(torch, ctx, bits, nbytes, samples):
    seed = 860 + len(bits) + nbytes % 7
    keys = inputs.make_keys(bits, seed)
    msg = inputs.make_message(nbytes, seed)
    km = inputs.random_map(len(msg), bits, seed)
    rblk = inputs.make_blinding(keys, km, seed)
    print(f"[gpu] blinded, bits {bits}, {len(km)} chunks", flush=True)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        assert len(rblk) == plan.ct_len
        cs, cr = plan.encrypt_blinded(dev(torch, msg), dev(torch, rblk))
        assert plan.check() == binding.PMK_OK
        pt = plan.decrypt_blinded(cs, cr)
        assert plan.check() == binding.PMK_OK
        cs_h = cs[: plan.ct_len].cpu().numpy()
        cr_h = cr[: plan.ct_len].cpu().numpy()
        pt_h = pt[: len(msg)].cpu().numpy()
    finally:
        plan.close()
    assert (pt_h == msg).all(), "blinded round trip differs"
    T = oracle.KeyTable(keys)
    spans = chunk_spans(keys, km, len(msg))
    rng = np.random.default_rng(seed)
    pick = np.unique(np.concatenate([rng.choice(len(km), min(samples, len(km)), replace=False), [len(km) - 1]]))
    for i in pick.tolist():
        mo, ln, co, kb = spans[i]
        k = int(km[i])
        m = int.from_bytes(bytes(msg[mo:mo + ln]), "big")
        r = int.from_bytes(bytes(rblk[co:co + kb]), "big")
        c_star, c_r = oracle.blind_int(T, k, "enc", m, r)
        assert bytes(cs_h[co:co + kb]) == c_star.to_bytes(kb, "big"), f"c* of chunk {i}"
        assert bytes(cr_h[co:co + kb]) == c_r.to_bytes(kb, "big"), f"c_R of chunk {i}"
        m2, r2 = oracle.blind_int(T, k, "dec", c_star, c_r)
        assert m2 == m and r2 == r


def test_blinded_flags_non_invertible_factor(torch, ctx):
    bits = [1024, 1024]
    keys = inputs.make_keys(bits, 870)
    msg = inputs.make_message(124 * 4, 870)
    km = inputs.round_robin_map(len(msg), bits)
    rblk = inputs.make_blinding(keys, km, 870)
    # chunk 2 (key 0): r = p, which shares a prime with N
    p = keys[0].p
    rblk[2 * 128:3 * 128] = np.frombuffer(p.to_bytes(128, "big"), np.uint8)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        cs, cr = plan.encrypt_blinded(dev(torch, msg), dev(torch, rblk))
        assert plan.check() == binding.PMK_OK
        pt = plan.decrypt_blinded(cs, cr)
        assert plan.check() == binding.PMK_EBLIND
        pt_h = pt[: len(msg)].cpu().numpy()
    finally:
        plan.close()
    # the other chunks are unaffected
    for i in (0, 1, 3):
        assert (pt_h[i * 124:(i + 1) * 124] == msg[i * 124:(i + 1) * 124]).all()


def test_blinding_factor_one_is_plain_rsa(torch, ctx):
    bits = [2048, 512]
    keys = inputs.make_keys(bits, 871)
    msg = inputs.make_message(3000, 871)
    km = inputs.random_map(len(msg), bits, 871)
    ones = []
    for k in km.tolist():
        kb = keys[k].bits // 8
        ones.append(np.frombuffer((1).to_bytes(kb, "big"), np.uint8))
    rblk = np.concatenate(ones)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        cs, cr = plan.encrypt_blinded(dev(torch, msg), dev(torch, rblk))
        ct = plan.encrypt(dev(torch, msg))
        assert plan.check() == binding.PMK_OK
        assert (cs[: plan.ct_len].cpu().numpy() == ct[: plan.ct_len].cpu().numpy()).all()  # c* = m^e
        assert (cr[: plan.ct_len].cpu().numpy() == rblk).all()                             # c_R = 1
    finally:
        plan.close()
