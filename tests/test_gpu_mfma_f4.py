"""GPU parity of the fp4 (e2m1) matrix-core contraction (shared seed).

0 and 1 are exact e2m1 values and fp32 sums of 0/1 products are exact
integers below 2^24, so the fp4 kernel must give the same bits as the oracle
and as the int8 and bit-sliced kernels."""

import numpy as np
import pytest

from tests.gpu_util import bit, first_diff, to_dev, to_dev_u32, to_host
from workloads import bernoulli_bits, permutation, uniform_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02856_amd import ssbh
    c = ssbh.Context(0)
    yield c
    c.close()


def hash_k(ctx, kern, sub, ln, wo, ns, seed, seed_bits, cap, **kw):
    import torch
    from paper_2308_02856_amd import ssbh
    out, tot, st = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed, seed_bits,
                                  cap, kernel=kern, **kw)
    torch.cuda.synchronize()
    assert int(st.item()) == 0, ssbh.status_name(int(st.item()))
    return to_host(out), int(tot.item())


@pytest.mark.parametrize("n,ns,m", [(4096, 256, 2048), (1024, 130, 1000),
                                    (3000, 33, 777), (65, 1, 64),
                                    (10000, 128, 4096), (2049, 64, 2049)])
def test_equal_blocks_match_oracle_int8_and_valu(ctx, orc, n, ns, m):
    from paper_2308_02856_amd import ssbh
    N = n * ns
    a = uniform_bits(N, n + ns + 3)
    perm = permutation(N, m + 3)
    sub, ln, wo, st = ctx.sample(to_dev(a), N, ns, ssbh.SAMPLE_PERMUTE,
                                 assign=to_dev_u32(perm))
    seed_bits = n + m - 1
    seed = to_dev(uniform_bits(seed_bits, 9 + m))
    kw = dict(out_rule=ssbh.OUT_FIXED, out_a=m)
    g4, t4 = hash_k(ctx, ssbh.K_MFMA_F4, sub, ln, wo, ns, seed, seed_bits, m, **kw)
    g8, t8 = hash_k(ctx, ssbh.K_MFMA_I8, sub, ln, wo, ns, seed, seed_bits, m, **kw)
    gv, tv = hash_k(ctx, ssbh.K_VALU, sub, ln, wo, ns, seed, seed_bits, m, **kw)
    osub, oln, owo, _ = orc.sample(a, N, ns, orc.SAMPLE_PERMUTE, assign=perm)
    want, wtot = orc.hash_batch(osub, oln, owo, np.full(ns, m, np.uint64),
                                to_host(seed), seed_bits, 0, m)
    assert t4 == t8 == tv == wtot
    assert np.array_equal(g4[: want.size], want), first_diff(g4[: want.size], want)
    assert np.array_equal(g4, g8) and np.array_equal(g4, gv)


@pytest.mark.parametrize("N,ns", [((1 << 20) + 999, 300), (200000, 7),
                                  (1 << 18, 1)])
def test_uneven_blocks_match_oracle(ctx, orc, N, ns):
    from paper_2308_02856_amd import ssbh
    a = bernoulli_bits(N, 0.3, N % 997)
    key = 0x4F4 + ns
    sub, ln, wo, st = ctx.sample(to_dev(a), N, ns, ssbh.SAMPLE_IID, key=key)
    osub, oln, owo, _ = orc.sample(a, N, ns, orc.SAMPLE_IID, key=key)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 2, 5)
    cap = int(om.max()) + 37
    seed_bits = int(oln.max()) + cap - 1 + 5
    seed = uniform_bits(seed_bits, 31)
    got, tot = hash_k(ctx, ssbh.K_MFMA_F4, sub, ln, wo, ns, to_dev(seed),
                      seed_bits, cap, out_rule=ssbh.OUT_RATIO, out_a=2, out_b=5)
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed, seed_bits, 0, cap)
    assert tot == wtot
    assert np.array_equal(got[: want.size], want), first_diff(got[: want.size], want)


def test_empty_and_short_blocks(ctx, orc):
    import torch
    from paper_2308_02856_amd import ssbh
    lens = [0, 1, 31, 32, 33, 0, 500, 64, 63, 65, 127, 128, 129] * 15
    ns = len(lens)
    words = [(L + 63) // 64 for L in lens]
    wo = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    sub = uniform_bits(64 * max(1, int(sum(words))), 15)
    for j, L in enumerate(lens):
        if L % 64:
            sub[int(wo[j]) + words[j] - 1] &= np.uint64((1 << (L % 64)) - 1)
    m = 45
    seed_bits = max(lens) + m - 1
    seed = uniform_bits(seed_bits, 16)
    ln_d = torch.tensor(lens, dtype=torch.int64, device="cuda")
    got, _ = hash_k(ctx, ssbh.K_MFMA_F4, to_dev(sub), ln_d, to_dev(wo), ns,
                    to_dev(seed), seed_bits, m, out_rule=ssbh.OUT_FIXED, out_a=m)
    want, _ = orc.hash_batch(sub, np.array(lens, np.uint64), wo,
                             np.full(ns, m, np.uint64), seed, seed_bits, 0, m)
    assert np.array_equal(got[: want.size], want)


@pytest.mark.parametrize("sched", [(8, 2, 4), (4, 4, 4), (4, 2, 4), (4, 2, 8),
                                   (8, 1, 4)])
@pytest.mark.parametrize("ksplit", [0, 1, 2, 3])
def test_every_schedule_and_k_split(ctx, orc, sched, ksplit):
    """Uneven i.i.d. sub-blocks of ~2^14 bits (several K chunks, ragged
    ends, chunks with an odd number of column words), every schedule and K
    split, against the oracle."""
    import torch
    from paper_2308_02856_amd import ssbh
    N, ns = (1 << 20) + 4321, 70
    a = bernoulli_bits(N, 0.4, 818)
    key = 0x77AB
    sub, ln, wo, st = ctx.sample(to_dev(a), N, ns, ssbh.SAMPLE_IID, key=key)
    osub, oln, owo, _ = orc.sample(a, N, ns, orc.SAMPLE_IID, key=key)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 3, 7)
    cap = int(om.max())
    seed_bits = int(oln.max()) + cap - 1
    seed = uniform_bits(seed_bits, 819)
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed, seed_bits, 0, cap)
    ctx.set_mfma_schedule(*sched, ksplit)
    try:
        out, tot, st2 = ctx.hash_batch(sub, sub.numel(), ln, wo, ns,
                                       to_dev(seed), seed_bits, cap,
                                       out_rule=ssbh.OUT_RATIO, out_a=3, out_b=7,
                                       kernel=ssbh.K_MFMA_F4)
        torch.cuda.synchronize()
        used = ctx.last_schedule()
    finally:
        ctx.set_mfma_schedule(0, 0, 0, 0)
    assert int(st2.item()) == 0 and int(tot.item()) == wtot
    assert used == "mfma4:%d:%d:%d:%d" % (*sched, ksplit)
    got = to_host(out)[: want.size]
    assert np.array_equal(got, want), first_diff(got, want)


def test_contraction_shape_equals_int8(ctx, orc):
    """2048 equal sub-blocks of 2^17 bits to 2^16 bits with one seed: fp4 ==
    int8 in full, sampled rows == the oracle."""
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns, m = 1 << 17, 2048, 1 << 16
    a = uniform_bits(n * ns, 87)
    ln = torch.full((ns,), n, dtype=torch.int64, device="cuda")
    wo = torch.arange(ns, dtype=torch.int64, device="cuda") * (n // 64)
    seed_bits = n + m - 1
    seed = uniform_bits(seed_bits, 88)
    kw = dict(out_rule=ssbh.OUT_FIXED, out_a=m)
    d_a, d_s = to_dev(a), to_dev(seed)
    g4, _ = hash_k(ctx, ssbh.K_MFMA_F4, d_a, ln, wo, ns, d_s, seed_bits, m, **kw)
    g8, _ = hash_k(ctx, ssbh.K_MFMA_I8, d_a, ln, wo, ns, d_s, seed_bits, m, **kw)
    assert np.array_equal(g4, g8), first_diff(g4, g8)
    rng = np.random.default_rng(55)
    for _ in range(100):
        j = int(rng.integers(0, ns))
        r = int(rng.integers(0, m))
        want = orc.toeplitz_rowwin(a[j * (n // 64):(j + 1) * (n // 64)], n,
                                   seed, seed_bits, 0, m, r)
        assert bit(g4, j * m + r) == want, (j, r)


def test_rejects_independent_seeds_and_inexact_lengths(ctx):
    import torch
    from paper_2308_02856_amd import ssbh
    x = to_dev(uniform_bits(128, 1))
    ln = torch.tensor([128, 128], dtype=torch.int64, device="cuda")
    wo = torch.tensor([0, 1], dtype=torch.int64, device="cuda")
    seed = to_dev(uniform_bits(1000, 2))
    with pytest.raises(ssbh.SsbhError) as e:
        ctx.hash_batch(x, 2, ln, wo, 2, seed, 1000, 64, out_rule=ssbh.OUT_FIXED,
                       out_a=64, seed_stride=200, kernel=ssbh.K_MFMA_F4)
    assert e.value.status == ssbh.E_INVAL
    big = to_dev(uniform_bits((1 << 24) + 200, 3))
    with pytest.raises(ssbh.SsbhError) as e:
        ctx.hash_batch(x, 2, ln, wo, 2, big, (1 << 24) + 200, 64,
                       out_rule=ssbh.OUT_FIXED, out_a=64, kernel=ssbh.K_MFMA_F4)
    assert e.value.status == ssbh.E_UNSUPPORTED
