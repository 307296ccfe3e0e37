"""GPU primality tests (key generation) against the oracle's Miller-Rabin and
trial division, exactly, with the same bases; and keys built from GPU-tested
primes run through the encryption path."""
import numpy as np
import pytest

import oracle
from paper_2111_11924_amd import binding, inputs, keygen

pytestmark = pytest.mark.gpu

STRONG_PSP_BASE2 = [2047, 3277, 4033, 4681, 8321, 15841, 29341, 42799, 49141, 52633]
CARMICHAEL = [561, 1105, 1729, 2465, 2821, 6601, 8911]


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    c = binding.Context(0)
    c.load_keys(inputs.make_keys([1024], 900))
    yield c
    c.close()


def words(x, n):
    return np.frombuffer(int(x).to_bytes(4 * n, "little"), dtype=np.uint32)


def candidates(bits, seed):
    rng = np.random.default_rng(seed)
    half = bits // 2
    out = list(STRONG_PSP_BASE2) + CARMICHAEL
    mers = [(1 << k) - 1 for k in (61, 89, 107, 127, 521, 607, 1279) if k <= half]
    out += mers
    g = np.random.Generator(np.random.PCG64(seed))
    primes = [inputs.gen_prime(half, g) for _ in range(3)]
    mask = (1 << half) - 1
    out += primes + [(primes[0] * primes[1]) & mask | 1, (primes[1] * primes[2] >> (half // 2)) & mask | 1]
    for _ in range(150):  # random odd numbers of the full candidate size
        out.append(inputs.rand_int(g, half) | 1 | (1 << (half - 1)))
    return out


@pytest.mark.parametrize("bits", [1024, 2048, 3072])
def test_miller_rabin_matches_oracle(torch, ctx, bits):
    nw = bits // 64
    cands = candidates(bits, 910 + bits)
    g = np.random.Generator(np.random.PCG64(920 + bits))
    rounds = 3
    bases = []
    for m in cands:  # base 2 first (the pseudoprimes pass it), then random bases
        bases.append([2] + [2 + inputs.rand_int(g, m.bit_length() + 32) % (m - 3) for _ in range(rounds - 1)])
    print(f"[gpu] Miller-Rabin, {bits}-bit keys, {len(cands)} candidates", flush=True)
    d_c = torch.from_numpy(np.concatenate([words(m, nw) for m in cands])).to("cuda")
    d_b = torch.from_numpy(np.concatenate([words(a, nw) for bs in bases for a in bs])).to("cuda")
    d_r = torch.full((len(cands),), 7, dtype=torch.int32, device="cuda")
    binding.pmk_miller_rabin(ctx.handle, bits, d_c, len(cands), d_b, rounds, d_r)
    got = d_r.cpu().numpy().tolist()
    want = [int(oracle.miller_rabin(m, bs)) for m, bs in zip(cands, bases)]
    assert got == want
    # the fixed facts behind it
    assert all(got[i] == 0 for i in range(len(STRONG_PSP_BASE2), len(STRONG_PSP_BASE2) + len(CARMICHAEL)))
    # base 2 alone lets the strong pseudoprimes through
    n = len(STRONG_PSP_BASE2)
    d_b2 = torch.from_numpy(np.concatenate([words(2, nw) for _ in range(n)])).to("cuda")
    d_r2 = torch.zeros(n, dtype=torch.int32, device="cuda")
    binding.pmk_miller_rabin(ctx.handle, bits, d_c, n, d_b2, 1, d_r2)
    assert d_r2.cpu().numpy().tolist() == [1] * n


@pytest.mark.parametrize("bits", [1024, 2048, 4096])
def test_sieve_matches_oracle(torch, ctx, bits):
    nw = bits // 64
    g = np.random.Generator(np.random.PCG64(930 + bits))
    cands = [inputs.rand_int(g, bits // 2) | 1 | (1 << (bits // 2 - 1)) for _ in range(300)]
    cands += [4093 * 4091 * 3, inputs.gen_prime(bits // 2, g)]
    d_c = torch.from_numpy(np.concatenate([words(m, nw) for m in cands])).to("cuda")
    d_f = torch.full((len(cands),), 7, dtype=torch.int32, device="cuda")
    binding.pmk_sieve(ctx.handle, bits, d_c, len(cands), d_f)
    assert d_f.cpu().numpy().tolist() == [int(oracle.trial_division_pass(m)) for m in cands]


def test_unsupported_sizes_are_refused(torch, ctx):
    buf = torch.zeros(64, dtype=torch.int32, device="cuda")
    with pytest.raises(binding.PmkError) as ei:
        binding.pmk_sieve(ctx.handle, 1536, buf, 1, buf)
    assert ei.value.status == binding.PMK_EUNSUPPORTED


def test_gpu_generated_keys_work(torch, ctx):
    keys = keygen.gpu_make_keys(ctx, 1024, 3, 940, rounds=20)
    for k in keys:
        assert binding.pmk_key_check(k) == (binding.PMK_OK, "")
        assert oracle.miller_rabin(k.p, [2, 3, 5, 7]) and oracle.miller_rabin(k.q, [2, 3, 5, 7])
    msg = inputs.make_message(3000, 940)
    km = inputs.round_robin_map(len(msg), [1024] * 3)
    ctx.load_keys(keys)
    plan = ctx.plan(km, len(msg))
    try:
        d_ct = plan.encrypt(torch.from_numpy(msg).to("cuda"))
        d_pt = plan.decrypt(d_ct)
        assert plan.check() == binding.PMK_OK
        ct = d_ct[: plan.ct_len].cpu().numpy()
        pt = d_pt[: len(msg)].cpu().numpy()
    finally:
        plan.close()
    assert (pt == msg).all()
    assert (ct == oracle.encrypt(oracle.KeyTable(keys), msg, km)).all()
