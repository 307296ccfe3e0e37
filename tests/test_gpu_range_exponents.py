"""GPU parity of the range rules of decryption, of public exponents of every
shape, of persistent launches whose waves each take several work units, and
of the mixed 25 MiB workload in full through the batched path.

Every comparison is exact (integer arithmetic).  Expected values come from the
CPU oracle; the oracle's decryption writes a chunk whose block is not below N
(a ciphertext lies in Z_N, Sec. 1.1) or whose plaintext is wider than the
chunk as zero bytes and reports -3, and the GPU must agree byte for byte and
report PMK_ERANGE.
"""
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2111_11924_amd import binding, inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def fixture_keys():
    with open(os.path.join(GOLDEN, "large_keys.json")) as f:
        return {k["bits"]: inputs.RsaKey.from_json(k) for k in json.load(f)["keys"]}


def spans(keys, km, msg_len):
    """(msg_off, len, ct_off, kb) of every chunk."""
    out, off, ct = [], 0, 0
    for k in km.tolist():
        kb = keys[k].bits // 8
        ln = min(kb - 4, msg_len - off)
        out.append((off, ln, ct, kb))
        off += ln
        ct += kb
    return out


# ---------------------------------------------------------------- range rules

def test_decrypt_range_rules_match_oracle(torch, ctx):
    """Blocks equal to N, above N, below N but decrypting wider than the chunk
    (random blocks, N - 1), a ragged last chunk whose plaintext needs one more
    byte than it has, and untouched blocks: the plain and the batched path
    write exactly the oracle's bytes and report PMK_ERANGE."""
    bits = [512, 2048, 4096, 1024]
    keys = inputs.make_keys(bits, 880)
    msg = inputs.make_message(30_000 + 3, 880)
    km = inputs.random_map(len(msg), bits, 880)
    T = oracle.KeyTable(keys)
    ct = oracle.encrypt(T, msg, km)
    sp = spans(keys, km, len(msg))
    rng = np.random.default_rng(880)
    bad = ct.copy()
    picks = rng.choice(len(km) - 1, 40, replace=False)
    for j, i in enumerate(picks.tolist()):
        mo, ln, co, kb = sp[i]
        n = keys[int(km[i])].n
        kind = j % 4
        if kind == 0:
            v = n
        elif kind == 1:
            v = (1 << (8 * kb)) - 1 - j
        elif kind == 2:
            v = n - 1
        else:
            v = int(rng.integers(1, 1 << 62)) * (n >> 64) % n
        bad[co:co + kb] = np.frombuffer(v.to_bytes(kb, "big"), np.uint8)
    # the last chunk: a plaintext one byte wider than its length
    mo, ln, co, kb = sp[-1]
    k = int(km[-1])
    c = oracle.rsa_int(T, k, "enc", 1 << (8 * ln))
    bad[co:co + kb] = np.frombuffer(c.to_bytes(kb, "big"), np.uint8)
    ref, rc = oracle.decrypt(T, bad, len(msg), km)
    assert rc == -3
    print(f"[gpu] range rules, {len(km)} chunks", flush=True)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        for batch in (False, True):
            out = torch.full((len(msg),), 0xA5, dtype=torch.uint8, device="cuda")
            plan.decrypt(dev(torch, bad), out, batch=batch)
            assert plan.check() == binding.PMK_ERANGE
            got = host(out, len(msg))
            diff = np.nonzero(got != ref)[0]
            assert len(diff) == 0, f"batch={batch}: differs at byte {diff[0]}"
        # the untouched ciphertext decrypts without a flag
        out = plan.decrypt(dev(torch, ct))
        assert plan.check() == binding.PMK_OK
        assert (host(out, len(msg)) == msg).all()
        # whole blocks: only the blocks >= N are rejected; every other block is m in full
        plan.set_decrypt_output(binding.PMK_DEC_BLOCKS)
        out = plan.decrypt(dev(torch, bad))
        assert plan.check() == binding.PMK_ERANGE
        blocks = host(out, plan.ct_len)
    finally:
        plan.close()
    for i in list(picks.tolist()) + [len(km) - 1]:
        mo, ln, co, kb = sp[i]
        k = int(km[i])
        cv = int.from_bytes(bytes(bad[co:co + kb]), "big")
        want = 0 if cv >= keys[k].n else oracle.rsa_int(T, k, "crt", cv)
        assert bytes(blocks[co:co + kb]) == want.to_bytes(kb, "big"), f"block {i}"


# ---------------------------------------------------------------- public exponents

SMALL_E = (3, 5, 7, 11, 13, 17, 19, 23)
TWO_WORD_E = ((1 << 33) + 1, (1 << 35) + (1 << 17) + 1, (1 << 40) + (1 << 20) + 1, (1 << 47) + 3)
DENSE_E = ((1 << 64) - 59, (1 << 64) - 83, (1 << 64) - 95, (1 << 64) - 179)


def with_exponent(base, cands):
    """base's primes with the first candidate e invertible modulo lambda(N)."""
    for e in cands:
        try:
            return inputs.key_from_primes(base.p, base.q, e, base.bits)
        except ValueError:
            continue
    raise AssertionError("no candidate exponent fits")


def base_keys(bits, count):
    if bits >= 2048:
        k = fixture_keys()[bits]
        return [k] * count
    return inputs.make_keys([bits] * count, 890 + bits // 64)


@pytest.mark.parametrize("bits", [128, 256, 512, 1024, 2048, 3072, 4096, 6144, 8192])
def test_public_exponents_of_every_shape(torch, ctx, bits):
    """e = a small prime (top bit 1 or 2), a sparse two-word e (33-48 bits) and a
    dense 64-bit e, through the one-lane and lane-group encryption kernels, the
    batched work queue (3072/4096 bits) and blinded encryption."""
    bases = base_keys(bits, 2)
    keys = [with_exponent(b, c) for c in (SMALL_E, TWO_WORD_E, DENSE_E) for b in bases]
    assert keys[0].e < 32 and keys[2].e >> 32 and keys[4].e >> 63
    kb = bits // 8
    nch = 64 * 2 + 23
    msg = inputs.make_message((nch - 1) * (kb - 4) + 5, 891 + bits)
    km = inputs.round_robin_map(len(msg), [bits] * len(keys))
    T = oracle.KeyTable(keys)
    ref_ct = oracle.encrypt(T, msg, km)
    rblk = inputs.make_blinding(keys, km, 892)
    print(f"[gpu] public exponents, {bits} bits, {len(km)} chunks", flush=True)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        d_msg = dev(torch, msg)
        ct_plain = host(plan.encrypt(d_msg), plan.ct_len)
        d_ct = plan.encrypt(d_msg, batch=True)
        ct_batch = host(d_ct, plan.ct_len)
        pt = host(plan.decrypt(d_ct), len(msg))
        cs, cr = plan.encrypt_blinded(d_msg, dev(torch, rblk))
        assert plan.check() == binding.PMK_OK
        cs_h, cr_h = host(cs, plan.ct_len), host(cr, plan.ct_len)
    finally:
        plan.close()
    assert (ct_plain == ref_ct).all() and (ct_batch == ref_ct).all()
    assert (pt == msg).all()
    sp = spans(keys, km, len(msg))
    for i in list(range(len(keys))) + [len(km) - 1]:  # one chunk of every key, and the last
        mo, ln, co, kb_ = sp[i]
        k = int(km[i])
        m = int.from_bytes(bytes(msg[mo:mo + ln]), "big")
        r = int.from_bytes(bytes(rblk[co:co + kb_]), "big")
        c_star, c_r = oracle.blind_int(T, k, "enc", m, r)
        assert bytes(cs_h[co:co + kb_]) == c_star.to_bytes(kb_, "big"), f"c* of chunk {i}"
        assert bytes(cr_h[co:co + kb_]) == c_r.to_bytes(kb_, "big"), f"c_R of chunk {i}"


# ---------------------------------------------------------------- several units per wave

def test_waves_take_several_units(torch, ctx):
    """With the persistent grids capped at a few waves, every exponentiation
    kernel -- encryption, CRT halves, the batched work queue, blinded
    decryption -- walks many work units per wave; results stay the oracle's."""
    bits = [512, 1024, 2048, 3072, 4096, 256]
    keys = inputs.make_keys(bits, 893)
    msg = inputs.make_message(80_000 + 9, 893)
    km = inputs.random_map(len(msg), bits, 893)
    T = oracle.KeyTable(keys)
    ref_ct = oracle.encrypt(T, msg, km)
    rblk = inputs.make_blinding(keys, km, 893)
    print(f"[gpu] capped grids, {len(km)} chunks", flush=True)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        for cap in (3, 7):
            ctx.set_grid_limit(cap)
            d_msg = dev(torch, msg)
            for batch in (False, True):
                d_ct = plan.encrypt(d_msg, batch=batch)
                ct = host(d_ct, plan.ct_len)
                pt = host(plan.decrypt(d_ct, batch=batch), len(msg))
                assert plan.check() == binding.PMK_OK
                assert (ct == ref_ct).all(), f"cap {cap}, batch {batch}: ciphertext"
                assert (pt == msg).all(), f"cap {cap}, batch {batch}: plaintext"
            cs, cr = plan.encrypt_blinded(d_msg, dev(torch, rblk))
            pt = host(plan.decrypt_blinded(cs, cr), len(msg))
            assert plan.check() == binding.PMK_OK
            assert (pt == msg).all(), f"cap {cap}: blinded"
    finally:
        ctx.set_grid_limit(0)
        plan.close()


# ---------------------------------------------------------------- lanes per number

def test_lane_forms_give_identical_bytes(torch, ctx):
    """CRT halves of the one-lane classes with 1, 2 or 4 lanes per number in a
    launch's short last round: with the grids uncapped (every launch here is
    one short round) and capped at 8 waves (full rounds of one lane per number,
    then a short round in lane groups), plain, batched and blinded (the
    one-chain blinded kernel and its lane-group form), every form gives the
    message back."""
    bits = [128, 256, 512, 1024, 2048, 3072, 4096, 768]
    keys = inputs.make_keys(bits, 895)
    msg = inputs.make_message(120_000 + 5, 895)
    km = inputs.random_map(len(msg), bits, 895)
    T = oracle.KeyTable(keys)
    ct = oracle.encrypt(T, msg, km)
    rblk = inputs.make_blinding(keys, km, 896)
    print(f"[gpu] lane forms, {len(km)} chunks", flush=True)
    ctx.load_keys(keys)
    classes = sorted(set(bits) - {768})
    default = {b: ctx.lanes(b) for b in classes + [8192]}
    plan = ctx.plan(km, len(msg))
    try:
        cs, cr = plan.encrypt_blinded(dev(torch, msg), dev(torch, rblk))
        assert plan.check() == binding.PMK_OK
        for lanes in (1, 2, 4):
            for b in classes:
                ctx.set_lanes(b, lanes, lanes)
            for cap in (0, 8):
                ctx.set_grid_limit(cap)
                for batch in (False, True):
                    pt = host(plan.decrypt(dev(torch, ct), batch=batch), len(msg))
                    assert plan.check() == binding.PMK_OK
                    assert (pt == msg).all(), f"lanes {lanes}, cap {cap}, batch {batch}"
                pt = host(plan.decrypt_blinded(cs, cr), len(msg))
                assert plan.check() == binding.PMK_OK
                assert (pt == msg).all(), f"blinded, lanes {lanes}, cap {cap}"
        with pytest.raises(binding.PmkError) as ei:
            ctx.set_lanes(6144, 2)
        assert ei.value.status == binding.PMK_EUNSUPPORTED
        ctx.set_lanes(8192, 4)  # its own form is accepted, and 8 lanes for small launches
        ctx.set_lanes(8192, 8, 4)
        with pytest.raises(binding.PmkError) as ei:
            ctx.set_lanes(8192, 8, 8)  # the tail form stays at 4
        assert ei.value.status == binding.PMK_EUNSUPPORTED
        with pytest.raises(binding.PmkError) as ei:
            ctx.set_lanes(1024, 8, 4)  # 8 only at 2048-4096 bits
        assert ei.value.status == binding.PMK_EUNSUPPORTED
        with pytest.raises(binding.PmkError) as ei:
            ctx.set_lanes(2048, 8, 8)  # and not for the tail form
        assert ei.value.status == binding.PMK_EUNSUPPORTED
        ctx.set_lanes(2048, 8, 2)
        ctx.set_lanes(8192, 4, 4)
        with pytest.raises(binding.PmkError) as ei:
            ctx.set_lanes(2048, 3)
        assert ei.value.status == binding.PMK_EINVAL
    finally:
        ctx.set_grid_limit(0)
        for b in default:
            ctx.set_lanes(b, *default[b])
        plan.close()


# ---------------------------------------------------------------- the mixed workload in full

def test_config3_full_size_batched(torch, ctx):
    """The mixed 25 MiB workload (256 keys of 1024-4096 bits, 81,570 chunks):
    the batched path's ciphertext equals the oracle's in full, it decrypts the
    oracle's ciphertext back to the message in full, and 1,024 sampled chunks
    per modulus size also through the oracle's CRT decryption."""
    w = inputs.config(3)
    keys, msg, km = w.keys(), w.message(), w.key_map()
    T = oracle.KeyTable(keys)
    print(f"[gpu] mixed 25 MiB workload, {len(km)} chunks: oracle encryption", flush=True)
    ref_ct = oracle.encrypt(T, msg, km)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        print("[gpu] batched encrypt / decrypt", flush=True)
        d_ct = plan.encrypt(dev(torch, msg), batch=True)
        ct = host(d_ct, plan.ct_len)
        pt = host(plan.decrypt(dev(torch, ref_ct), batch=True), len(msg))
        assert plan.check() == binding.PMK_OK
    finally:
        plan.close()
    diff = np.nonzero(ct != ref_ct)[0]
    assert len(diff) == 0, f"ciphertext differs at byte {diff[0]} ({len(diff)} bytes)"
    diff = np.nonzero(pt != msg)[0]
    assert len(diff) == 0, f"plaintext differs at byte {diff[0]}"
    # sampled chunks through the oracle's own CRT decryption, as one sub-message
    sp = spans(keys, km, len(msg))
    sizes = np.array([k.bits for k in keys])[km]
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([rng.choice(np.nonzero(sizes == b)[0], 1024, replace=False)
                                    for b in (1024, 2048, 3072, 4096)] + [[len(km) - 1]]))
    sub_m = np.concatenate([msg[sp[i][0]:sp[i][0] + sp[i][1]] for i in idx.tolist()]).astype(np.uint8)
    sub_c = np.concatenate([ct[sp[i][2]:sp[i][2] + sp[i][3]] for i in idx.tolist()]).astype(np.uint8)
    print(f"[gpu] oracle CRT decryption of {len(idx)} sampled chunks", flush=True)
    sub_pt, rc = oracle.decrypt(T, sub_c, len(sub_m), km[idx])
    assert rc == 0 and (sub_pt == sub_m).all()
