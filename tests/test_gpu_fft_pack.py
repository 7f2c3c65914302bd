"""GPU parity of the FFT hash with four sub-blocks per transform (each part
x_lo + 2^18 x_hi) against two per transform and the oracle: bit for bit,
tolerance 0, including ragged last transforms, the largest values packing
admits, and the refusal when sub-blocks could reach 2^18 bits."""

import numpy as np
import pytest

from tests.gpu_util import first_diff, to_dev, to_host
from workloads import bernoulli_bits, uniform_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02856_amd import ssbh
    c = ssbh.Context(0)
    yield c
    c.close()


def fft_hash(ctx, per_part, sub, ln, wo, ns, seed, seed_bits, cap, **kw):
    import torch
    from paper_2308_02856_amd import ssbh
    ctx.set_fft_packing(per_part)
    try:
        out, tot, st = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed,
                                      seed_bits, cap, kernel=ssbh.K_FFT, **kw)
        torch.cuda.synchronize()
        sched = ctx.last_schedule()
    finally:
        ctx.set_fft_packing(0)
    assert int(st.item()) == 0, ssbh.status_name(int(st.item()))
    return to_host(out), int(tot.item()), sched


@pytest.mark.parametrize("N,ns", [((1 << 20) + 999, 300), (200000, 9),
                                  (5000, 64), (1 << 17, 1), (3 * (1 << 16) + 5, 7),
                                  (40000, 6)])
def test_two_and_four_per_transform_match_oracle(ctx, orc, N, ns):
    from paper_2308_02856_amd import ssbh
    a = bernoulli_bits(N, 0.4, N % 997 + ns)
    key = 0x5eed + ns
    sub, ln, wo, _ = ctx.sample(to_dev(a), N, ns, ssbh.SAMPLE_IID, key=key)
    osub, oln, owo, _ = orc.sample(a, N, ns, orc.SAMPLE_IID, key=key)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 2, 5)
    cap = int(om.max()) + 5
    seed_bits = int(oln.max()) + cap - 1 + 2
    seed = uniform_bits(seed_bits, 31 + ns)
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed, seed_bits, 0, cap)
    kw = dict(out_rule=ssbh.OUT_RATIO, out_a=2, out_b=5)
    for per_part in (1, 2):
        got, tot, sched = fft_hash(ctx, per_part, sub, ln, wo, ns, to_dev(seed),
                                   seed_bits, cap, **kw)
        assert ":x%d:" % (2 * per_part) in sched, sched
        assert tot == wtot
        assert np.array_equal(got[: want.size], want), (per_part, first_diff(got[: want.size], want))


def test_library_packs_short_sub_blocks_only(ctx):
    """Library choice: four per transform for short sub-blocks and L <= 2^20,
    two when a sub-block may reach 2^18 bits."""
    from paper_2308_02856_amd import ssbh
    N, ns = 1 << 16, 8
    a = uniform_bits(N, 3)
    sub, ln, wo, _ = ctx.sample(to_dev(a), N, ns, ssbh.SAMPLE_IID, key=9)
    nmax = int(ln.max().item())
    kw = dict(out_rule=ssbh.OUT_FIXED, out_a=100)
    for extra, per in ((0, 4), ((1 << 18) - nmax, 2)):
        seed_bits = nmax + 100 - 1 + extra
        seed = to_dev(uniform_bits(seed_bits, 4))
        _, _, sched = fft_hash(ctx, 0, sub, ln, wo, ns, seed, seed_bits, 100, **kw)
        assert ":x%d:" % per in sched, sched


def test_packed_extreme_magnitudes(ctx):
    """All-one sub-blocks up to 2^18 - 1 bits (the longest packing admits)
    and an all-one seed: every middle-product entry is n_j, so each part's
    integer n_lo + 2^18 n_hi is near 2^36, and every output bit is
    n_j mod 2.  Six sub-blocks: one full transform and a half one."""
    import torch
    from paper_2308_02856_amd import ssbh
    n = (1 << 18) - 1
    lens = np.array([n, n - 1, n - 2, n, n - 3, n - 6], dtype=np.uint64)
    m = 1 << 18
    words = (lens + 63) // 64
    wo = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    sub = np.full(int(words.sum()), np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    for j in range(len(lens)):            # clear the bits past n_j
        r = int(lens[j]) % 64
        if r:
            sub[int(wo[j] + words[j] - 1)] = np.uint64((1 << r) - 1)
    seed_bits = n + m - 1
    seed = np.full((seed_bits + 63) // 64, np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    seed[-1] = np.uint64((1 << (seed_bits % 64)) - 1)
    d_sub = to_dev(sub)
    d_ln = torch.from_numpy(lens.view(np.int64)).cuda()
    d_wo = torch.from_numpy(wo.view(np.int64)).cuda()
    got, tot, sched = fft_hash(ctx, 2, d_sub, d_ln, d_wo, len(lens), to_dev(seed),
                               seed_bits, m, out_rule=ssbh.OUT_FIXED, out_a=m)
    assert ":x4:" in sched and tot == m * len(lens)
    bits = np.unpackbits(got.view(np.uint8), bitorder="little")[: tot]
    for j in range(len(lens)):
        blk = bits[j * m:(j + 1) * m]
        assert np.all(blk == (int(lens[j]) & 1)), (j, int(blk.sum()))


def test_forced_packing_refused_for_long_sub_blocks(ctx):
    """Forcing four per transform when seed_bits + 1 - m_cap reaches 2^18
    (a sub-block could then reach 2^18 bits) is refused on the host."""
    from paper_2308_02856_amd import ssbh
    N, ns = 1 << 16, 4
    a = uniform_bits(N, 8)
    sub, ln, wo, _ = ctx.sample(to_dev(a), N, ns, ssbh.SAMPLE_IID, key=5)
    cap = 64
    seed_bits = (1 << 18) + cap - 1
    seed = to_dev(uniform_bits(seed_bits, 6))
    ctx.set_fft_packing(2)
    try:
        with pytest.raises(ssbh.SsbhError) as e:
            ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed, seed_bits, cap,
                           out_rule=ssbh.OUT_FIXED, out_a=cap, kernel=ssbh.K_FFT)
    finally:
        ctx.set_fft_packing(0)
    assert e.value.status == ssbh.E_UNSUPPORTED


@pytest.mark.parametrize("mode", ["two", "four", "stride"])
def test_degenerate_sub_blocks_every_layout(ctx, orc, mode):
    """Empty sub-blocks, m_j = 0, m_j = 1, m_j > n_j and outputs that start
    and end inside a word, for two and four sub-blocks per transform and for
    independent seeds (one per transform): the parity words go through the
    scratch layout and the emit pass in every case."""
    import torch
    from paper_2308_02856_amd import ssbh
    lens = np.array([0, 5, 64, 0, 1000, 3, 700, 65, 1, 130], dtype=np.uint64)
    outl = np.array([4, 0, 100, 0, 333, 9, 1, 64, 1, 63], dtype=np.uint64)
    words = (lens + 63) // 64
    wo = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    sub = uniform_bits(int(words.sum()) * 64, 12)
    for j in range(len(lens)):          # clear the bits past n_j
        r = int(lens[j]) % 64
        if r and words[j]:
            sub[int(wo[j] + words[j] - 1)] &= np.uint64((1 << r) - 1)
    ns = len(lens)
    cap = int(outl.max())
    stride = int(lens.max()) + cap - 1 + 7 if mode == "stride" else 0
    seed_bits = stride * ns if stride else int(lens.max()) + cap - 1
    seed = uniform_bits(seed_bits, 13)
    dl = torch.from_numpy(outl.view(np.int64)).cuda()
    per_part = {"two": 1, "four": 2, "stride": 0}[mode]
    got, tot, sched = fft_hash(ctx, per_part, to_dev(sub), to_dev(lens), to_dev(wo),
                               ns, to_dev(seed), seed_bits, cap,
                               out_rule=ssbh.OUT_EXPLICIT, out_len=dl, seed_stride=stride)
    assert ":x%d:" % {"two": 2, "four": 4, "stride": 1}[mode] in sched, sched
    want, wtot = orc.hash_batch(sub, lens, wo, outl, seed, seed_bits, stride, cap)
    assert tot == wtot
    assert np.array_equal(got[: want.size], want), first_diff(got[: want.size], want)
