"""GPU tests of the request server (continuous batching): every served result
equals the oracle's, alone and in a mix of concurrent requests; admission,
validation and device-detected errors are reported per request."""
import threading

import numpy as np
import pytest

import oracle
from paper_2111_11924_amd import binding, inputs

pytestmark = pytest.mark.gpu

BITS = [512, 1024, 2048, 3072, 4096, 768, 1536, 2048, 1024, 512, 3584, 256]


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def keys():
    return inputs.make_keys(BITS, 850)


@pytest.fixture(scope="module")
def table(keys):
    return oracle.KeyTable(keys)


@pytest.fixture()
def ctx(torch, keys):
    c = binding.Context(0)
    c.load_keys(keys)
    yield c
    c.close()


def make_requests(n, seed, max_len=40_000):
    """Small mixed requests (the oracle checks every byte)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        size = int(rng.integers(1, max_len))
        k = int(rng.integers(1, 6))
        subset = [int(x) for x in rng.choice(len(BITS), size=k, replace=False)]
        km = inputs.map_over_subset(size, subset, BITS)
        reqs.append((int(rng.random() < 0.5), inputs.make_message(size, seed * 1000 + i), km))
    return reqs


@pytest.mark.parametrize("depth", [1, 2])
def test_served_results_alone_and_in_the_mix(ctx, table, depth):
    reqs = make_requests(24, 851)
    # decryption inputs: the oracle's ciphertext of the request's message
    inputs_ = []
    for op, msg, km in reqs:
        ct = oracle.encrypt(table, msg, km)
        inputs_.append(ct if op == binding.PMK_OP_DECRYPT else msg)
    print(f"[gpu] server: {len(reqs)} requests", flush=True)
    srv = ctx.server(staging_bytes=8 << 20, round_chunks=2048, pipeline_depth=depth)
    try:
        # the first request alone
        op, msg, km = reqs[0]
        t, out = srv.submit(op, inputs_[0], len(msg), km)
        info = srv.wait(t)
        assert info["status"] == binding.PMK_OK and info["state"] == binding.PMK_REQ_DONE
        alone = out.copy()
        # all of them at once, from two submitting threads
        tickets = [None] * len(reqs)

        def submit(idx):
            for i in idx:
                op, msg, km = reqs[i]
                tickets[i] = srv.submit(op, inputs_[i], len(msg), km)

        th = [threading.Thread(target=submit, args=(range(j, len(reqs), 2),)) for j in range(2)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        outs = []
        for t, out in tickets:
            info = srv.wait(t)
            assert info["status"] == binding.PMK_OK
            assert info["t_submit_ns"] <= info["t_admit_ns"] <= info["t_done_ns"]
            outs.append(out)
        st = srv.stats()
        assert st["requests_done"] == len(reqs) + 1 and st["rounds"] >= 2
    finally:
        srv.stop()
    assert (outs[0] == alone).all(), "a request's result changed when served in the mix"
    for (op, msg, km), out in zip(reqs, outs):
        if op == binding.PMK_OP_ENCRYPT:
            assert (out == oracle.encrypt(table, msg, km)).all()
        else:
            assert (out == msg).all()


def test_admission_queues_requests_beyond_staging(ctx, table):
    # a slab that holds only a few requests at a time: the rest queue
    reqs = make_requests(12, 852, max_len=30_000)
    srv = ctx.server(staging_bytes=256 << 10, round_chunks=512)
    try:
        tickets = []
        for op, msg, km in reqs:
            data = oracle.encrypt(table, msg, km) if op == binding.PMK_OP_DECRYPT else msg
            tickets.append(srv.submit(op, data, len(msg), km))
        for (op, msg, km), (t, out) in zip(reqs, tickets):
            assert srv.wait(t)["status"] == binding.PMK_OK
            if op == binding.PMK_OP_DECRYPT:
                assert (out == msg).all()
            else:
                assert (out == oracle.encrypt(table, msg, km)).all()
        # a request larger than the whole slab is refused at submission
        big = inputs.make_message(300_000, 852)
        km = inputs.map_over_subset(len(big), [2], BITS)
        with pytest.raises(binding.PmkError) as ei:
            srv.submit(binding.PMK_OP_ENCRYPT, big, len(big), km)
        assert ei.value.status == binding.PMK_ESIZE
    finally:
        srv.stop()


def test_errors_are_per_request(ctx, keys, table):
    srv = ctx.server()
    try:
        msg = inputs.make_message(5000, 853)
        km = inputs.map_over_subset(len(msg), [1, 2], BITS)
        bad = km.copy()
        bad[0] = len(BITS)
        with pytest.raises(binding.PmkError) as ei:
            srv.submit(binding.PMK_OP_ENCRYPT, msg, len(msg), bad)
        assert ei.value.status == binding.PMK_EKEY
        with pytest.raises(binding.PmkError) as ei:
            srv.submit(binding.PMK_OP_ENCRYPT, msg, len(msg), km, out=np.zeros(10, np.uint8))
        assert ei.value.status == binding.PMK_ESIZE
        # the key table and windows are frozen while the server runs
        with pytest.raises(binding.PmkError) as ei:
            ctx.load_keys(keys)
        assert ei.value.status == binding.PMK_EBUSY
        with pytest.raises(binding.PmkError) as ei:
            ctx.set_window(2048, 4)
        assert ei.value.status == binding.PMK_EBUSY
        # a ciphertext block equal to its modulus fails that request only
        ct = oracle.encrypt(table, msg, km)
        broken = ct.copy()
        nb = keys[1].bits // 8
        broken[:nb] = np.frombuffer(keys[1].n.to_bytes(nb, "big"), np.uint8)
        t_bad, out_bad = srv.submit(binding.PMK_OP_DECRYPT, broken, len(msg), km)
        # a block below its modulus whose plaintext is wider than the chunk
        # (N - 1 decrypts to itself) fails its request too, in the same round
        wide = ct.copy()
        nb2 = keys[int(km[1])].bits // 8
        off2 = nb
        wide[off2:off2 + nb2] = np.frombuffer((keys[int(km[1])].n - 1).to_bytes(nb2, "big"), np.uint8)
        t_wide, out_wide = srv.submit(binding.PMK_OP_DECRYPT, wide, len(msg), km)
        t_ok, out_ok = srv.submit(binding.PMK_OP_DECRYPT, ct, len(msg), km)
        assert srv.wait(t_bad)["status"] == binding.PMK_ERANGE
        assert srv.wait(t_wide)["status"] == binding.PMK_ERANGE
        assert srv.wait(t_ok)["status"] == binding.PMK_OK
        assert (out_ok == msg).all()
        # the rejected chunks are zeros, the rest decrypted: the oracle's bytes
        for data, out in ((broken, out_bad), (wide, out_wide)):
            ref, rc = oracle.decrypt(table, data, len(msg), km)
            assert rc == -3 and (out == ref).all()
        # an empty request completes at once
        t_e, out_e = srv.submit(binding.PMK_OP_ENCRYPT, np.zeros(0, np.uint8), 0, np.zeros(0, np.uint32))
        assert srv.wait(t_e)["status"] == binding.PMK_OK and len(out_e) == 0
        with pytest.raises(binding.PmkError):
            srv.wait(t_e)  # forgotten once reported done
    finally:
        srv.stop()
    rc, _ = binding.pmk_submit(ctx.handle, 0, msg, np.zeros(64, np.uint8), len(msg), km)
    assert rc == binding.PMK_EINVAL  # no server any more
    ctx.load_keys(keys)  # allowed again
