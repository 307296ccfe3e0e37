"""GPU parity of the host-buffer forms (pmk_encrypt_host / pmk_decrypt_host):
the paper's transfer / compute / merge pipeline (Sec. 3.3) over slices of the
chunk range, from pinned and from pageable host memory, against the oracle
byte for byte."""
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


@pytest.mark.parametrize("slices", [0, 1, 3, 7])
def test_host_forms_match_oracle(torch, ctx, slices):
    bits = [1024, 2048, 512, 3072]
    keys = inputs.make_keys(bits, 960)
    msg = inputs.make_message(200_000 + 7, 960)
    km = inputs.random_map(len(msg), bits, 960)
    T = oracle.KeyTable(keys)
    ref_ct = oracle.encrypt(T, msg, km)
    print(f"[gpu] host forms, {slices} slices, {len(km)} chunks", flush=True)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        # pinned buffers (torch pin_memory)
        h_msg = torch.from_numpy(msg.copy()).pin_memory()
        h_ct = torch.zeros(plan.ct_len, dtype=torch.uint8).pin_memory()
        h_pt = torch.zeros(len(msg), dtype=torch.uint8).pin_memory()
        assert plan.encrypt_host(h_msg, h_ct, slices) == binding.PMK_OK
        assert (h_ct.numpy() == ref_ct).all()
        assert plan.decrypt_host(h_ct, h_pt, slices) == binding.PMK_OK
        assert (h_pt.numpy() == msg).all()
        # pageable numpy buffers, a second call on the same slices
        ct2 = np.zeros(plan.ct_len, np.uint8)
        pt2 = np.zeros(len(msg), np.uint8)
        assert plan.encrypt_host(msg, ct2, slices) == binding.PMK_OK
        assert plan.decrypt_host(ref_ct, pt2, slices) == binding.PMK_OK
        assert (ct2 == ref_ct).all() and (pt2 == msg).all()
        # an out-of-range block: PMK_ERANGE and the oracle's bytes
        bad = ref_ct.copy()
        kb0 = keys[int(km[0])].bits // 8
        bad[:kb0] = np.frombuffer(keys[int(km[0])].n.to_bytes(kb0, "big"), np.uint8)
        pt3 = np.zeros(len(msg), np.uint8)
        assert plan.decrypt_host(bad, pt3, slices) == binding.PMK_ERANGE
        ref3, rc = oracle.decrypt(T, bad, len(msg), km)
        assert rc == -3 and (pt3 == ref3).all()
        # whole blocks out
        plan.set_decrypt_output(binding.PMK_DEC_BLOCKS)
        blocks = np.zeros(plan.ct_len, np.uint8)
        assert plan.decrypt_host(ref_ct, blocks, slices) == binding.PMK_OK
    finally:
        plan.close()
    # every block is its chunk's plaintext, left-padded to the block size
    off = ct = 0
    for k in km.tolist():
        kb = keys[k].bits // 8
        ln = min(kb - 4, len(msg) - off)
        assert int.from_bytes(bytes(blocks[ct:ct + kb]), "big") == int.from_bytes(bytes(msg[off:off + ln]), "big")
        off += ln
        ct += kb


def test_host_decryption_cut_at_whole_rounds(torch, ctx):
    """Default slicing of a decryption whose key map allows cuts at whole rounds
    of CRT work (one size class, round-robin over 16 keys: every slice gives
    each key full tiles): 1 and 2 rounds then the rest -- the same bytes as
    one slice and as the device form, a block of every slice against the oracle,
    and an out-of-range block in the last slice flagged."""
    keys = [k for k in inputs.make_keys([2048] * 16, 962)]
    nch = 3 * 98_304 + 5_000  # slices of 1 and 2 rounds of the 3,072-wave chip, then the rest
    kb = 256
    msg = inputs.make_message((nch - 1) * (kb - 4) + 17, 962)
    km = inputs.round_robin_map(len(msg), [2048] * 16)
    assert len(km) == nch
    T = oracle.KeyTable(keys)
    print(f"[gpu] host decryption at whole rounds, {nch} chunks", flush=True)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        d_ct = plan.encrypt(torch.from_numpy(msg).to("cuda"))
        ct = d_ct[: plan.ct_len].cpu().numpy()
        pt0 = np.zeros(len(msg), np.uint8)
        pt1 = np.zeros(len(msg), np.uint8)
        assert plan.decrypt_host(ct, pt0, 0) == binding.PMK_OK
        assert plan.decrypt_host(ct, pt1, 1) == binding.PMK_OK
        assert (pt0 == msg).all() and (pt1 == msg).all()
        bad = ct.copy()
        bad[-kb:] = np.frombuffer(keys[int(km[-1])].n.to_bytes(kb, "big"), np.uint8)
        pt2 = np.zeros(len(msg), np.uint8)
        assert plan.decrypt_host(bad, pt2, 0) == binding.PMK_ERANGE
        assert (pt2[:-17] == msg[:-17]).all() and (pt2[-17:] == 0).all()
    finally:
        plan.close()
    # a chunk on each side of the slice boundaries (1 and 3 rounds) against the oracle's encryption
    for i in (0, 98_303, 98_304, 294_911, 294_912, nch - 1):
        k = int(km[i])
        m = int.from_bytes(bytes(msg[i * (kb - 4):min((i + 1) * (kb - 4), len(msg))]), "big")
        assert int.from_bytes(bytes(ct[i * kb:(i + 1) * kb]), "big") == oracle.rsa_int(T, k, "enc", m)


def test_host_forms_empty_and_errors(torch, ctx):
    keys = inputs.make_keys([512], 961)
    ctx.load_keys(keys)
    plan = ctx.plan(np.zeros(0, np.uint32), 0)
    try:
        assert plan.encrypt_host(np.zeros(4, np.uint8), np.zeros(4, np.uint8)) == binding.PMK_OK
    finally:
        plan.close()
    msg = inputs.make_message(500, 961)
    km = inputs.round_robin_map(500, [512])
    plan = ctx.plan(km, len(msg))
    try:
        assert binding.pmk_encrypt_host(plan.handle, None, np.zeros(plan.ct_len, np.uint8), 0) == binding.PMK_EINVAL
    finally:
        plan.close()
