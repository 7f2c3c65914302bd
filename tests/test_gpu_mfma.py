"""GPU parity of the int8 matrix-core contraction (shared seed).

The contraction computes the same Toeplitz hashes as the bit-sliced kernel
whenever all sub-blocks share one seed; it is compared with the oracle and
bit for bit with the bit-sliced (VALU) kernel on the same inputs.
"""

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


@pytest.fixture(scope="module")
def S():
    from paper_2308_02856_amd import ssbh
    return ssbh


def run_both(ctx, S, sub, ln, wo, ns, seed, seed_bits, cap, **kw):
    import torch
    outs = []
    for kern in (S.K_MFMA_I8, S.K_VALU):
        out, tot, st = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed,
                                      seed_bits, cap, kernel=kern, **kw)
        torch.cuda.synchronize()
        assert int(st.item()) == 0, (kern, S.status_name(int(st.item())))
        outs.append((to_host(out), int(tot.item())))
    return outs


@pytest.mark.parametrize("n,ns,m", [(4096, 256, 2048), (1024, 130, 1000),
                                    (3000, 33, 777), (65, 1, 64),
                                    (10000, 128, 4096)])
def test_equal_blocks_match_oracle_and_valu(ctx, S, orc, n, ns, m):
    N = n * ns
    a = uniform_bits(N, n + ns)
    perm = permutation(N, m)
    sub, ln, wo, st = ctx.sample(to_dev(a), N, ns, S.SAMPLE_PERMUTE,
                                 assign=to_dev_u32(perm))
    seed_bits = n + m - 1
    seed = uniform_bits(seed_bits, 7 + m)
    (g_mfma, t1), (g_valu, t2) = run_both(
        ctx, S, sub, ln, wo, ns, to_dev(seed), seed_bits, m,
        out_rule=S.OUT_FIXED, out_a=m)
    osub, oln, owo, _ = orc.sample(a, N, ns, orc.SAMPLE_PERMUTE, assign=perm)
    want, wtot = orc.hash_batch(osub, oln, owo, np.full(ns, m, np.uint64),
                                seed, seed_bits, 0, m)
    assert t1 == t2 == wtot
    assert np.array_equal(g_mfma[: want.size], want), first_diff(g_mfma[: want.size], want)
    assert np.array_equal(g_mfma, g_valu)


@pytest.mark.parametrize("N,ns", [((1 << 20) + 999, 300), (200000, 7),
                                  (1 << 18, 1)])
def test_uneven_blocks_match_oracle_and_valu(ctx, S, orc, N, ns):
    a = bernoulli_bits(N, 0.3, N % 1000)
    key = 0x1234 + ns
    sub, ln, wo, st = ctx.sample(to_dev(a), N, ns, S.SAMPLE_IID, key=key)
    osub, oln, owo, _ = orc.sample(a, N, ns, orc.SAMPLE_IID, key=key)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 2, 5)
    cap = int(om.max()) + 37          # cap above every m_j
    seed_bits = int(oln.max()) + cap - 1 + 5
    seed = uniform_bits(seed_bits, 3)
    (g_mfma, t1), (g_valu, t2) = run_both(
        ctx, S, sub, ln, wo, ns, to_dev(seed), seed_bits, cap,
        out_rule=S.OUT_RATIO, out_a=2, out_b=5)
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed, seed_bits, 0, cap)
    assert t1 == t2 == wtot
    assert np.array_equal(g_mfma[: want.size], want), first_diff(g_mfma[: want.size], want)
    assert np.array_equal(g_mfma, g_valu)


def test_empty_and_short_blocks(ctx, S, orc):
    import torch
    lens = [0, 1, 31, 32, 33, 0, 500, 64, 63] * 20
    ns = len(lens)
    words = [(L + 63) // 64 for L in lens]
    wo = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    sub = uniform_bits(64 * max(1, int(sum(words))), 5)
    for j, L in enumerate(lens):
        if L % 64:
            sub[int(wo[j]) + words[j] - 1] &= np.uint64((1 << (L % 64)) - 1)
    m = 45
    seed_bits = max(lens) + m - 1
    seed = uniform_bits(seed_bits, 6)
    ln_d = torch.tensor(lens, dtype=torch.int64, device="cuda")
    (g_mfma, _), (g_valu, _) = run_both(
        ctx, S, to_dev(sub), ln_d, to_dev(wo), ns, to_dev(seed), seed_bits, m,
        out_rule=S.OUT_FIXED, out_a=m)
    want, _ = orc.hash_batch(sub, np.array(lens, np.uint64), wo,
                             np.full(ns, m, np.uint64), seed, seed_bits, 0, m)
    assert np.array_equal(g_mfma[: want.size], want)
    assert np.array_equal(g_mfma, g_valu)


def test_mfma_rejects_independent_seeds(ctx, S):
    import torch
    x = to_dev(uniform_bits(128, 1))
    ln = torch.tensor([128, 128], dtype=torch.int64, device="cuda")
    wo = torch.tensor([0, 1], dtype=torch.int64, device="cuda")
    with pytest.raises(S.SsbhError):
        ctx.hash_batch(x, 2, ln, wo, 2, to_dev(uniform_bits(1000, 2)), 1000,
                       64, out_rule=S.OUT_FIXED, out_a=64, seed_stride=200,
                       kernel=S.K_MFMA_I8)


def test_contraction_shape_sampled_rows(ctx, S, orc):
    """2048 equal sub-blocks of 2^17 bits hashed to 2^16 bits each with one
    seed (the contraction workload's shape on a quarter of its sub-blocks):
    MFMA == VALU in full, and 300 sampled rows against the oracle."""
    import torch
    n, ns, m = 1 << 17, 2048, 1 << 16
    N = n * ns
    a = uniform_bits(N, 77)
    ln = torch.full((ns,), n, dtype=torch.int64, device="cuda")
    wo = torch.arange(ns, dtype=torch.int64, device="cuda") * (n // 64)
    seed_bits = n + m - 1
    seed = uniform_bits(seed_bits, 78)
    (g_mfma, t1), (g_valu, t2) = run_both(
        ctx, S, to_dev(a), ln, wo, ns, to_dev(seed), seed_bits, m,
        out_rule=S.OUT_FIXED, out_a=m)
    assert t1 == t2 == n * ns // 2
    assert np.array_equal(g_mfma, g_valu), first_diff(g_mfma, g_valu)
    rng = np.random.default_rng(5)
    for _ in range(300):
        j = int(rng.integers(0, ns))
        r = int(rng.integers(0, m))
        want = orc.toeplitz_rowwin(a[j * (n // 64):(j + 1) * (n // 64)], n,
                                   seed, seed_bits, 0, m, r)
        assert bit(g_mfma, j * m + r) == want, (j, r)


SCHEDULES = [(8, 2, 4), (4, 4, 4), (4, 2, 4), (4, 2, 8), (8, 1, 4)]


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("ksplit", [0, 1, 2, 3, 5])
def test_every_schedule_and_k_split(ctx, S, orc, sched, ksplit):
    """Every matrix-core schedule and K split (partial parities merged by
    XOR) gives the oracle's bits: uneven i.i.d. sub-blocks of ~2^14 bits
    (several K chunks of 2048 columns, ragged ends), output segments at
    arbitrary bit offsets, m_j spanning several 32-row words and row tiles."""
    import torch
    N, ns = (1 << 20) + 4321, 70
    a = bernoulli_bits(N, 0.4, 808)
    key = 0x77AA
    sub, ln, wo, st = ctx.sample(to_dev(a), N, ns, S.SAMPLE_IID, key=key)
    osub, oln, owo, _ = orc.sample(a, N, ns, orc.SAMPLE_IID, key=key)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 3, 7)
    cap = int(om.max())
    seed_bits = int(oln.max()) + cap - 1
    seed = uniform_bits(seed_bits, 809)
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed, seed_bits, 0, cap)
    ctx.set_mfma_schedule(*sched, ksplit)
    try:
        out, tot, st2 = ctx.hash_batch(sub, sub.numel(), ln, wo, ns,
                                       to_dev(seed), seed_bits, cap,
                                       out_rule=S.OUT_RATIO, out_a=3, out_b=7,
                                       kernel=S.K_MFMA_I8)
        torch.cuda.synchronize()
        used = ctx.last_schedule()
    finally:
        ctx.set_mfma_schedule(0, 0, 0, 0)
    assert int(st2.item()) == 0 and int(tot.item()) == wtot
    assert used == "mfma:%d:%d:%d:%d" % (*sched, ksplit)
    got = to_host(out)[: want.size]
    assert np.array_equal(got, want), first_diff(got, want)


def test_k_split_beyond_chunks_is_exact(ctx, S, orc):
    """More K splits than K chunks: empty splits contribute nothing."""
    import torch
    n, ns, m = 3000, 40, 2500          # 2 chunks of 2048 columns
    N = n * ns
    a = uniform_bits(N, 91)
    perm = permutation(N, 92)
    sub, ln, wo, st = ctx.sample(to_dev(a), N, ns, S.SAMPLE_PERMUTE,
                                 assign=to_dev_u32(perm))
    seed_bits = n + m - 1
    seed = uniform_bits(seed_bits, 93)
    ctx.set_mfma_schedule(8, 2, 4, 7)
    try:
        out, tot, st2 = ctx.hash_batch(sub, sub.numel(), ln, wo, ns,
                                       to_dev(seed), seed_bits, m,
                                       out_rule=S.OUT_FIXED, out_a=m,
                                       kernel=S.K_MFMA_I8)
        torch.cuda.synchronize()
    finally:
        ctx.set_mfma_schedule(0, 0, 0, 0)
    osub, oln, owo, _ = orc.sample(a, N, ns, orc.SAMPLE_PERMUTE, assign=perm)
    want, _ = orc.hash_batch(osub, oln, owo, np.full(ns, m, np.uint64), seed,
                             seed_bits, 0, m)
    assert int(st2.item()) == 0
    assert np.array_equal(to_host(out)[: want.size], want)
