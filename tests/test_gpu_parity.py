"""GPU parity: the HIP path against the CPU oracle, byte for byte.

Every comparison is exact (integer arithmetic: tolerance 0).  Sizes span
several 64-chunk tiles per size class plus a ragged last tile; the 100 MiB
workload is checked on sampled chunks against the oracle and in full through
the decrypt(encrypt(m)) = m identity (Sec. 1.1 correctness of RSA).
"""
import json
import os
from concurrent.futures import ThreadPoolExecutor
from functools import lru_cache

import numpy as np
import pytest

import oracle
from paper_2111_11924_amd import binding, inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@lru_cache(maxsize=1)
def fixture_keys():
    """The seeded 2048-8192-bit key pairs stored in tests/golden/large_keys.json."""
    with open(os.path.join(GOLDEN, "large_keys.json")) as f:
        return {k["bits"]: inputs.RsaKey.from_json(k) for k in json.load(f)["keys"]}


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


def host(t, n):
    return t[:n].cpu().numpy()


def gpu_roundtrip(torch, ctx, keys, msg, km):
    """(ciphertext, decrypted) from the GPU, decrypting the GPU's own ciphertext."""
    print(f"[gpu] {len(keys)} keys, {len(msg)} bytes, {len(km)} chunks", flush=True)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        d_msg = dev(torch, msg)
        d_ct = plan.encrypt(d_msg)
        assert plan.check() == binding.PMK_OK
        ct = host(d_ct, plan.ct_len)
        d_pt = plan.decrypt(d_ct)
        assert plan.check() == binding.PMK_OK
        pt = host(d_pt, len(msg))
    finally:
        plan.close()
    return ct, pt


def check_against_oracle(torch, ctx, keys, msg, km):
    T = oracle.KeyTable(keys)
    ct, pt = gpu_roundtrip(torch, ctx, keys, msg, km)
    ref_ct = oracle.encrypt(T, msg, km)
    assert len(ct) == len(ref_ct)
    bad = np.nonzero(ct != ref_ct)[0]
    assert len(bad) == 0, f"ciphertext differs at byte {bad[0]} ({len(bad)} bytes)"
    ref_pt, rc = oracle.decrypt(T, ref_ct, len(msg), km, crt=True)
    assert rc == 0 and (ref_pt == msg).all()
    bad = np.nonzero(pt != msg)[0]
    assert len(bad) == 0, f"plaintext differs at byte {bad[0]} ({len(bad)} bytes)"


def test_config1_small_512bit(torch, ctx):
    w = inputs.config(1)
    check_against_oracle(torch, ctx, w.keys(), w.message(), w.key_map())


@pytest.mark.parametrize("bits", [128, 256, 512, 1024, 2048, 3072, 4096])
def test_each_size_class_several_tiles_ragged(torch, ctx, bits):
    keys = inputs.make_keys([bits] * 5, 700 + bits)
    kb = bits // 8
    nch = 64 * 3 + 17  # several tiles per key and a ragged last tile
    msg_len = (nch - 1) * (kb - 4) + 3  # last chunk: 3 bytes
    msg = inputs.make_message(msg_len, bits)
    km = inputs.round_robin_map(msg_len, [bits] * 5)
    assert len(km) == nch
    check_against_oracle(torch, ctx, keys, msg, km)


def test_mixed_sizes_random_map(torch, ctx):
    # sizes that are not class sizes run in the next class up
    bits = [128, 512, 2048, 256, 1024, 768, 192, 1536, 384, 2048, 3072, 4096, 2560, 3584]
    keys = inputs.make_keys(bits, 801)
    msg = inputs.make_message(150_000 + 7, 801)
    km = inputs.random_map(len(msg), bits, 801)
    check_against_oracle(torch, ctx, keys, msg, km)


def test_special_chunk_values(torch, ctx):
    bits = [512, 1024]
    keys = inputs.make_keys(bits, 802)
    caps = [b // 8 - 4 for b in bits]
    parts = [
        np.zeros(caps[0], np.uint8),                                   # m = 0
        np.concatenate([np.zeros(caps[1] - 1, np.uint8), [1]]),        # m = 1
        np.full(caps[0], 0xFF, np.uint8),                              # largest chunk value
        np.concatenate([np.zeros(caps[1] - 2, np.uint8), [1, 0]]),     # leading zero bytes
        np.concatenate([[0x80], np.zeros(caps[0] - 1, np.uint8)]),
        np.array([7], np.uint8),                                       # 1-byte last chunk
    ]
    msg = np.concatenate(parts).astype(np.uint8)
    km = np.array([0, 1, 0, 1, 0, 1], np.uint32)
    T = oracle.KeyTable(keys)
    ct, pt = gpu_roundtrip(torch, ctx, keys, msg, km)
    assert (ct == oracle.encrypt(T, msg, km)).all()
    assert (pt == msg).all()
    # m = 0 and m = 1 are fixed points
    assert not ct[:64].any()
    assert ct[64:192].tolist() == [0] * 127 + [1]


def test_decrypt_of_zero_and_one_blocks(torch, ctx):
    keys = inputs.make_keys([1024], 803)
    msg_len = 2 * 124
    km = np.zeros(2, np.uint32)
    ct = np.zeros(256, np.uint8)
    ct[255] = 1  # block 0 = 0, block 1 = 1
    ctx.load_keys(keys)
    plan = ctx.plan(km, msg_len)
    try:
        d_pt = plan.decrypt(dev(torch, ct))
        assert plan.check() == binding.PMK_OK
        pt = host(d_pt, msg_len)
    finally:
        plan.close()
    ref, rc = oracle.decrypt(oracle.KeyTable(keys), ct, msg_len, km)
    assert rc == 0 and (pt == ref).all()
    assert not pt[:124].any() and pt[124:].tolist() == [0] * 123 + [1]


def test_block_not_below_modulus_is_reported(torch, ctx):
    keys = inputs.make_keys([512, 512], 804)
    msg = inputs.make_message(600, 804)
    km = inputs.round_robin_map(600, [512, 512])
    T = oracle.KeyTable(keys)
    ct = oracle.encrypt(T, msg, km)
    bad = ct.copy()
    bad[64:128] = np.frombuffer(keys[1].n.to_bytes(64, "big"), np.uint8)  # block 1 = N
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        d_pt = plan.decrypt(dev(torch, bad))
        assert plan.check() == binding.PMK_ERANGE
        pt = host(d_pt, len(msg))
        assert plan.check() == binding.PMK_OK  # the flag was cleared
    finally:
        plan.close()
    assert (pt[:60] == msg[:60]).all() and (pt[120:] == msg[120:]).all()
    assert not pt[60:120].any()  # the rejected chunk is written as zeros
    ref, rc = oracle.decrypt(T, bad, len(msg), km)
    assert rc == -3 and (pt == ref).all()


def test_empty_message(torch, ctx):
    keys = inputs.make_keys([512], 805)
    ctx.load_keys(keys)
    plan = ctx.plan(np.zeros(0, np.uint32), 0)
    try:
        assert plan.ct_len == 0
        buf = torch.zeros(4, dtype=torch.uint8, device="cuda")
        plan.encrypt(buf, buf)
        plan.decrypt(buf, buf)
        assert plan.check() == binding.PMK_OK
    finally:
        plan.close()


def test_one_shot_entry_points_and_errors(torch, ctx):
    keys = inputs.make_keys([1024, 1024], 806)
    msg = inputs.make_message(1000, 806)
    km = inputs.round_robin_map(1000, [1024, 1024])
    ctx.load_keys(keys)
    d_msg = dev(torch, msg)
    ct_len = 128 * len(km)
    d_ct = torch.empty(ct_len, dtype=torch.uint8, device="cuda")
    assert binding.pmk_encrypt(ctx.handle, d_msg, len(msg), km, d_ct, ct_len) == binding.PMK_OK
    assert binding.pmk_encrypt(ctx.handle, d_msg, len(msg), km, d_ct, ct_len - 1) == binding.PMK_ESIZE
    assert binding.pmk_encrypt(ctx.handle, d_msg, len(msg), km[:-1], d_ct, ct_len) == binding.PMK_ESIZE
    bad = km.copy()
    bad[0] = 9
    assert binding.pmk_encrypt(ctx.handle, d_msg, len(msg), bad, d_ct, ct_len) == binding.PMK_EKEY
    d_pt = torch.empty(len(msg), dtype=torch.uint8, device="cuda")
    assert binding.pmk_decrypt(ctx.handle, d_ct, ct_len, km, d_pt, len(msg)) == binding.PMK_OK
    assert (host(d_pt, len(msg)) == msg).all()
    assert (host(d_ct, ct_len) == oracle.encrypt(oracle.KeyTable(keys), msg, km)).all()
    # replacing keys while a plan is alive is refused
    plan = ctx.plan(km, len(msg))
    with pytest.raises(binding.PmkError) as ei:
        ctx.load_keys(keys)
    assert ei.value.status == binding.PMK_EBUSY
    plan.close()
    ctx.load_keys(keys)


def test_config2_1MiB_2048bit(torch, ctx):
    w = inputs.config(2)
    check_against_oracle(torch, ctx, w.keys(), w.message(), w.key_map())


def test_config4_100MiB_sampled_and_roundtrip(torch, ctx):
    w = inputs.config(4)
    keys, msg, km = w.keys(), w.message(), w.key_map()
    assert len(km) == 416_102
    ct, pt = gpu_roundtrip(torch, ctx, keys, msg, km)
    bad = np.nonzero(pt != msg)[0]
    assert len(bad) == 0, f"roundtrip differs at byte {bad[0]}"
    T = oracle.KeyTable(keys)
    rng = np.random.default_rng(4)
    sample = np.unique(np.concatenate([rng.choice(len(km), 200, replace=False), [0, 1, len(km) - 1]]))
    for i in sample.tolist():
        k = int(km[i])
        lo = i * 252
        m = int.from_bytes(bytes(msg[lo:lo + 252]), "big")
        c = oracle.rsa_int(T, k, "enc", m)
        assert bytes(ct[i * 256:(i + 1) * 256]) == c.to_bytes(256, "big"), i
        assert oracle.rsa_int(T, k, "crt", c) == m


# ---------------------------------------------------------------- batched path

def batch_roundtrip(torch, ctx, plan, msg, replays=3):
    """Encrypt + decrypt through the graph-captured batch entry points `replays`
    times, with unrelated eager work and synchronisations between replays;
    returns every replay's (ciphertext, plaintext)."""
    d_msg = dev(torch, msg)
    d_ct = torch.zeros(max(plan.ct_len, 4), dtype=torch.uint8, device="cuda")
    d_pt = torch.zeros(max(len(msg), 4), dtype=torch.uint8, device="cuda")
    outs = []
    for k in range(replays):
        d_ct.zero_()
        d_pt.fill_(0xA5)
        plan.encrypt(d_msg, d_ct, batch=True)
        plan.decrypt(d_ct, d_pt, batch=True)
        assert plan.check() == binding.PMK_OK
        outs.append((host(d_ct, plan.ct_len), host(d_pt, len(msg))))
        junk = torch.randn(1 << 16, device="cuda")  # eager work between replays
        torch.cuda.synchronize()
        del junk
    return outs


@pytest.mark.parametrize("bits", [
    [512, 1024, 2048, 3072, 4096, 256, 2048, 1024, 128, 3584],  # both batch groups + small classes
    [2048, 2048, 1024],                                         # one-lane classes only
    [4096, 3072],                                               # multi-lane classes only
    [256, 512],                                                 # small classes only
])
def test_batch_path_matches_oracle_every_replay(torch, ctx, bits):
    keys = inputs.make_keys(bits, 810 + len(bits))
    msg = inputs.make_message(60_000 + 13, 810)
    km = inputs.random_map(len(msg), bits, 810)
    print(f"[gpu] batch path, bits {bits}, {len(km)} chunks", flush=True)
    ctx.load_keys(keys)
    T = oracle.KeyTable(keys)
    ref_ct = oracle.encrypt(T, msg, km)
    plan = ctx.plan(km, len(msg))
    try:
        outs = batch_roundtrip(torch, ctx, plan, msg)
        # the plain path on the same plan gives the same bytes
        d_ct = plan.encrypt(dev(torch, msg))
        plain_ct = host(d_ct, plan.ct_len)
    finally:
        plan.close()
    assert (plain_ct == ref_ct).all()
    for k, (ct, pt) in enumerate(outs):
        assert (ct == ref_ct).all(), f"replay {k}: ciphertext differs"
        assert (pt == msg).all(), f"replay {k}: plaintext differs"


def test_batch_path_new_buffers_and_profiling(torch, ctx):
    bits = [1024, 4096, 2048]
    keys = inputs.make_keys(bits, 820)
    msg = inputs.make_message(20_000, 820)
    km = inputs.round_robin_map(len(msg), bits)
    ctx.load_keys(keys)
    ref_ct = oracle.encrypt(oracle.KeyTable(keys), msg, km)
    plan = ctx.plan(km, len(msg))
    try:
        d_msg = dev(torch, msg)
        for _ in range(2):  # fresh output buffers each time: the graph is recaptured
            d_ct = plan.encrypt(d_msg, batch=True)
            d_pt = plan.decrypt(d_ct, batch=True)
            assert plan.check() == binding.PMK_OK
            assert (host(d_ct, plan.ct_len) == ref_ct).all()
            assert (host(d_pt, len(msg)) == msg).all()
        plan.profile(True)
        d_ct = plan.encrypt(d_msg, batch=True)
        d_pt = plan.decrypt(d_ct, batch=True)
        ms, n = plan.kernel_time(binding.PMK_KERNEL_BATCH)
        plan.profile(False)
        assert n == 1 and ms > 0  # the work-queue launch of the 4096-bit encryption
        assert (host(d_ct, plan.ct_len) == ref_ct).all()
        assert (host(d_pt, len(msg)) == msg).all()
    finally:
        plan.close()


@pytest.mark.parametrize("win", [2, 3, 4, 6, 5])
def test_window_width_never_changes_results(torch, ctx, win):
    bits = [1024, 2048, 3072, 512]
    keys = inputs.make_keys(bits, 830)
    msg = inputs.make_message(40_000 + 1, 830)
    km = inputs.random_map(len(msg), bits, 830)
    ctx.load_keys(keys)
    default = {b: ctx.window(b) for b in bits}
    for b in bits:
        ctx.set_window(b, win)
        assert ctx.window(b) == win
    ref_ct = oracle.encrypt(oracle.KeyTable(keys), msg, km)
    plan = ctx.plan(km, len(msg))
    try:
        d_ct = dev(torch, ref_ct)
        for batch in (False, True):
            d_pt = plan.decrypt(d_ct, batch=batch)
            assert plan.check() == binding.PMK_OK
            assert (host(d_pt, len(msg)) == msg).all(), f"window {win}, batch {batch}"
    finally:
        plan.close()
        for b in bits:
            ctx.set_window(b, default[b])
    with pytest.raises(binding.PmkError):
        ctx.set_window(2048, 7)


def test_autotune_cache_and_results(torch, ctx, tmp_path):
    bits = [2048, 1024, 512, 6144]
    keys = inputs.make_keys(bits, 840)
    ctx.load_keys(keys)
    default = {b: ctx.window(b) for b in bits}
    default_lanes = {b: ctx.lanes(b) for b in bits}
    cache = str(tmp_path / "tune.txt")
    try:
        ctx.autotune(cache)
        lines = open(cache).read().splitlines()
        assert lines[0].startswith("pmk-autotune 2 ")
        chosen = {int(l.split()[0]): [int(x) for x in l.split()[1:4]] for l in lines[1:]}
        assert set(chosen) == set(bits)
        for b in bits:
            w, fill, tail = chosen[b]
            assert ctx.window(b) == w and ctx.lanes(b) == (fill, tail)
            assert w in ((4, 5, 6) if b >= 1024 else (3, 4, 5))
            if b >= 6144:  # lane-group class: its own 4 lanes, or 8 for small launches
                assert fill in (4, 8) and tail == 4
            else:  # 8 lanes for small launches at 2048-4096 bits
                assert fill in ((1, 2, 4, 8) if b >= 2048 else (1, 2, 4)) and tail in (1, 2, 4)
        # the cache is applied without measuring
        for b in bits:
            ctx.set_window(b, 2)
            ctx.set_lanes(b, *((4, 4) if b >= 6144 else (1, 1)))
        ctx.autotune(cache)
        assert all(ctx.window(b) == chosen[b][0] and ctx.lanes(b) == tuple(chosen[b][1:]) for b in bits)
        msg = inputs.make_message(30_000 + 3, 840)
        km = inputs.random_map(len(msg), bits, 840)
        check_against_oracle(torch, ctx, keys, msg, km)
    finally:
        for b in bits:
            ctx.set_window(b, default[b])
            ctx.set_lanes(b, *default_lanes[b])


# ---------------------------------------------------------------- 6144/8192-bit keys
# (the paper's largest key sizes: full-size numbers over 8 lanes, CRT halves over 4)

@pytest.mark.parametrize("bits", [6144, 8192])
def test_large_classes_several_tiles_ragged(torch, ctx, bits):
    keys = inputs.make_keys([bits] * 3, 700000 + bits)
    kb = bits // 8
    nch = 64 * 2 + 9  # several tiles per key, ragged last tile
    msg_len = (nch - 1) * (kb - 4) + 5
    msg = inputs.make_message(msg_len, bits)
    km = inputs.round_robin_map(msg_len, [bits] * 3)
    assert len(km) == nch
    T = oracle.KeyTable(keys)
    ct, pt = gpu_roundtrip(torch, ctx, keys, msg, km)
    assert (ct == oracle.encrypt(T, msg, km)).all()
    assert (pt == msg).all()
    for i in (0, 1, 64, nch - 1):  # CRT decryption of single blocks by the oracle
        k = int(km[i])
        c = int.from_bytes(bytes(ct[i * kb:(i + 1) * kb]), "big")
        m = int.from_bytes(bytes(msg[i * (kb - 4):(i + 1) * (kb - 4)]), "big")
        assert oracle.rsa_int(T, k, "crt", c) == m


def test_large_and_small_classes_mixed_batch_and_blinded(torch, ctx):
    bits = [6144, 8192, 5120, 2048, 1024]  # 5120 runs in the 6144-bit class
    keys = inputs.make_keys(bits, 890)
    msg = inputs.make_message(90_000 + 17, 890)
    km = inputs.random_map(len(msg), bits, 890)
    T = oracle.KeyTable(keys)
    ref_ct = oracle.encrypt(T, msg, km)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        outs = batch_roundtrip(torch, ctx, plan, msg, replays=2)
        rblk = inputs.make_blinding(keys, km, 890)
        cs, cr = plan.encrypt_blinded(dev(torch, msg), dev(torch, rblk))
        pt_b = plan.decrypt_blinded(cs, cr)
        assert plan.check() == binding.PMK_OK
        cs_h = host(cs, plan.ct_len)
        cr_h = host(cr, plan.ct_len)
        pt_bh = host(pt_b, len(msg))
    finally:
        plan.close()
    for k, (ct, pt) in enumerate(outs):
        assert (ct == ref_ct).all(), f"replay {k}"
        assert (pt == msg).all(), f"replay {k}"
    assert (pt_bh == msg).all()
    # one blinded chunk of each key against the oracle's blinding routine
    off = ct_off = 0
    seen = set()
    for i, k in enumerate(km.tolist()):
        kb = keys[k].bits // 8
        ln = min(kb - 4, len(msg) - off)
        if k not in seen and ln == kb - 4:
            seen.add(k)
            m = int.from_bytes(bytes(msg[off:off + ln]), "big")
            r = int.from_bytes(bytes(rblk[ct_off:ct_off + kb]), "big")
            c_star, c_r = oracle.blind_int(T, k, "enc", m, r)
            assert bytes(cs_h[ct_off:ct_off + kb]) == c_star.to_bytes(kb, "big")
            assert bytes(cr_h[ct_off:ct_off + kb]) == c_r.to_bytes(kb, "big")
        off += ln
        ct_off += kb
    assert len(seen) == len(bits)


# ---------------------------------------------------------------- exponent shapes
# The window schedule is read from the private exponents themselves.  Key
# material with CRT exponents of unusual shape -- zero, one, a single bit, zero
# runs longer than the 64 exponent bits a step reads ahead, a set bit only at
# the top -- is still a valid input to the CRT route (the unique m < N with
# m = C^dp mod p and m = C^dq mod q), so the GPU must match the oracle's CRT
# route bit for bit on every block.  Such blocks decrypt to values as wide as N,
# so the plan writes whole blocks (PMK_DEC_BLOCKS) and every bit is compared.

def _special_exponents(h):
    return [
        (0, 1),
        (1, 3),
        (1 << (h - 2), (1 << (h - 2)) | 1),
        ((1 << (h - 2)) | 1, (1 << 200) | (1 << 130) | 5),
        ((0b101101 << (h - 8)) | (1 << 65) | 1, (1 << 63) | (1 << 64)),
        ((1 << (h - 3)) - 1, 7 << 70),
    ]


def base_key(bits):
    """One key pair of the given size: the stored seeded keys for 2048 bits and
    up (large primes take minutes to find), generated below that."""
    if bits >= 2048:
        return fixture_keys()[bits]
    return inputs.make_keys([bits], 850 + bits // 64)[0]


def oracle_many(fn, jobs):
    """fn over jobs on the host cores (the oracle's calls release the GIL)."""
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(fn, jobs))


@pytest.mark.parametrize("bits,lanes", [(b, l) for b in (1024, 2048, 3072, 4096) for l in (1, 2, 4)]
                         + [(2048, 8), (3072, 8), (4096, 8), (6144, 4), (6144, 8), (8192, 4), (8192, 8)])
def test_unusual_crt_exponents(torch, ctx, bits, lanes):
    """(lanes: lanes per number of the CRT halves where the launch leaves the
    chip mostly idle -- here every launch, 6 keys x 70 chunks; 8 at 2048-4096
    bits; the 6144/8192-bit classes take 4, or 8 for such launches.)"""
    base = base_key(bits)
    h = bits // 2
    keys = []
    for dp, dq in _special_exponents(h):
        d = dict(base.__dict__)
        d.update(dp=dp % base.p, dq=dq % base.q)
        keys.append(inputs.RsaKey(**d))
    kb = bits // 8
    per_key = 70  # a full tile and a ragged one per key
    km = np.repeat(np.arange(len(keys), dtype=np.uint32), per_key)
    g = np.random.Generator(np.random.PCG64([851, bits]))
    ct = g.integers(0, 256, size=len(km) * kb, dtype=np.uint8)
    ct.reshape(-1, kb)[:, 0] = 0  # every block below N
    msg_len = len(km) * (kb - 4)
    print(f"[gpu] unusual CRT exponents, {bits} bits, {lanes} lanes, {len(km)} blocks", flush=True)
    ctx.load_keys(keys)
    default = ctx.lanes(bits)
    plan = ctx.plan(km, msg_len)
    T = oracle.KeyTable(keys)
    try:
        ctx.set_lanes(bits, lanes, min(lanes, 4))
        plan.set_decrypt_output(binding.PMK_DEC_BLOCKS)
        d_m = plan.decrypt(dev(torch, ct))
        assert plan.check() == binding.PMK_OK
        got = host(d_m, plan.ct_len)
    finally:
        ctx.set_lanes(bits, *default)
        plan.close()
    # every block up to 2048 bits; above, sampled blocks of every key
    # (first, second, last of the full tile, the ragged tile's first and last)
    rows = list(range(len(km))) if bits <= 2048 else \
        [k * per_key + j for k in range(len(keys)) for j in (0, 1, 63, 64, per_key - 1)]
    ref = oracle_many(lambda i: oracle.rsa_int(T, int(km[i]), "crt",
                                               int.from_bytes(bytes(ct[i * kb:(i + 1) * kb]), "big")), rows)
    for i, m in zip(rows, ref):
        assert bytes(got[i * kb:(i + 1) * kb]) == m.to_bytes(kb, "big"), f"block {i} (key {km[i]})"


@pytest.mark.parametrize("bits,lanes", [(b, l) for b in (1024, 2048, 3072, 4096) for l in (1, 2, 4)]
                         + [(2048, 8), (3072, 8), (4096, 8), (6144, 4), (6144, 8), (8192, 4), (8192, 8)])
def test_blinded_decryption_with_unusual_exponents(torch, ctx, bits, lanes):
    """Blinded decryption (c* and c_R in one squaring chain per prime) with
    private exponents of unusual shape: d below both primes, so dp = dq = d
    keeps the shape, and the second exponent p-1-d is dense.  Whole blocks
    against the oracle's blinded route m = (c*)^d (c_R^d)^-1 mod N, in every
    lanes-per-number form (the launch is under one round, so all of it runs
    in the form set)."""
    base = base_key(bits)
    h = bits // 2
    exps = [1, 3, (1 << 70) + 5, (1 << (h - 3)) - 1, (1 << (h - 2)) | 1, (1 << 100) | (1 << 37)]
    keys = []
    for d in exps:
        assert d < base.q - 1 and d < base.p - 1
        f = dict(base.__dict__)
        f.update(d=d, dp=d, dq=d)
        keys.append(inputs.RsaKey(**f))
    kb = bits // 8
    per_key = 66
    km = np.repeat(np.arange(len(keys), dtype=np.uint32), per_key)
    g = np.random.Generator(np.random.PCG64([852, bits]))
    cs = g.integers(0, 256, size=len(km) * kb, dtype=np.uint8)
    cr = g.integers(0, 256, size=len(km) * kb, dtype=np.uint8)
    cs.reshape(-1, kb)[:, 0] = 0
    cr.reshape(-1, kb)[:, 0] = 0
    msg_len = len(km) * (kb - 4)
    print(f"[gpu] blinded decryption, unusual exponents, {bits} bits, lanes {lanes}, {len(km)} blocks", flush=True)
    ctx.load_keys(keys)
    plan = ctx.plan(km, msg_len)
    T = oracle.KeyTable(keys)
    default = ctx.lanes(bits)
    try:
        ctx.set_lanes(bits, lanes, min(lanes, 4))
        plan.set_decrypt_output(binding.PMK_DEC_BLOCKS)
        d_m = plan.decrypt_blinded(dev(torch, cs), dev(torch, cr))
        assert plan.check() == binding.PMK_OK
        got = host(d_m, plan.ct_len)
    finally:
        ctx.set_lanes(bits, *default)
        plan.close()
    rows = [k * per_key + j for k in range(len(keys)) for j in (0, 1, 63, 64, per_key - 1)]

    def ref(i):
        c1 = int.from_bytes(bytes(cs[i * kb:(i + 1) * kb]), "big")
        c2 = int.from_bytes(bytes(cr[i * kb:(i + 1) * kb]), "big")
        return oracle.blind_int(T, int(km[i]), "dec", c1, c2)[0]

    for i, m in zip(rows, oracle_many(ref, rows)):
        assert bytes(got[i * kb:(i + 1) * kb]) == m.to_bytes(kb, "big"), f"block {i} (key {km[i]})"
