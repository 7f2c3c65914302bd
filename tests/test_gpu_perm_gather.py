"""GPU: the streaming gather of the permutation-split sampling (inputs of
2^26 bits and more: cells by source window, bits looked up from a window in
LDS, merged back by slot) gives the oracle's sub-blocks bit for bit, equals
the direct gather, falls back to the direct gather when a permutation
overfills a cell, and reports an out-of-range entry."""

import numpy as np
import pytest

from tests.gpu_util import first_diff, to_dev, to_dev_u32, to_host
from workloads import uniform_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02856_amd import ssbh
    c = ssbh.Context(0)
    yield c
    c.close()


def sample(ctx, a_dev, n, ns, perm=None, key=0, path=0):
    import torch
    from paper_2308_02856_amd import ssbh
    ctx.set_sample_path(path)
    try:
        if perm is None:
            r = ctx.sample(a_dev, n, ns, ssbh.SAMPLE_PERMUTE, key=key)
        else:
            r = ctx.sample(a_dev, n, ns, ssbh.SAMPLE_PERMUTE, assign=perm)
        torch.cuda.synchronize()
    finally:
        ctx.set_sample_path(0)
    return r


def test_keyed_streamed_gather_matches_oracle(ctx, orc):
    """2^26 bits, 64 sub-blocks, the library's keyed permutation."""
    n, ns, key = 1 << 26, 64, 0x26262626
    a = uniform_bits(n, 261)
    sub, ln, wo, st = sample(ctx, to_dev(a), n, ns, key=key)
    assert int(st.item()) == 0
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_PERMUTE,
                                   assign=orc.permutation(n, key))
    got = to_host(sub)[: osub.size]
    assert np.array_equal(got, osub), first_diff(got, osub)
    assert np.array_equal(to_host(ln)[:ns], oln)


def test_ragged_sub_blocks_random_permutation(ctx, orc):
    """n = 5 * 13421773 (sub-blocks of 13421773 bits, not whole words), a
    caller permutation: oracle equality and equality with the direct path."""
    n, ns = 5 * 13421773, 5
    a = uniform_bits(n, 262)
    perm = np.random.default_rng(263).permutation(n).astype(np.uint32)
    d_a, d_p = to_dev(a), to_dev_u32(perm)
    sub, _, _, st = sample(ctx, d_a, n, ns, perm=d_p)
    assert int(st.item()) == 0
    osub, _, _, _ = orc.sample(a, n, ns, orc.SAMPLE_PERMUTE, assign=perm)
    got = to_host(sub)[: osub.size]
    assert np.array_equal(got, osub), first_diff(got, osub)
    sub1, _, _, st1 = sample(ctx, d_a, n, ns, perm=d_p, path=1)
    assert int(st1.item()) == 0
    assert np.array_equal(to_host(sub1)[: osub.size], got)


@pytest.mark.parametrize("kind", ["identity", "reversed"])
def test_concentrated_permutation_falls_back(ctx, orc, kind):
    """Identity and reversal put a whole chunk into one window, far past a
    cell's capacity: the direct gather writes the output, bit-exact."""
    n, ns = 1 << 26, 16
    a = uniform_bits(n, 264)
    perm = np.arange(n, dtype=np.uint32)
    if kind == "reversed":
        perm = perm[::-1].copy()
    sub, _, _, st = sample(ctx, to_dev(a), n, ns, perm=to_dev_u32(perm))
    assert int(st.item()) == 0
    osub, _, _, _ = orc.sample(a, n, ns, orc.SAMPLE_PERMUTE, assign=perm)
    got = to_host(sub)[: osub.size]
    assert np.array_equal(got, osub), first_diff(got, osub)


def test_out_of_range_entry_is_reported(ctx):
    from paper_2308_02856_amd import ssbh
    n, ns = 1 << 26, 8
    a = uniform_bits(n, 265)
    perm = np.random.default_rng(266).permutation(n).astype(np.uint32)
    perm[12345] = n
    _, _, _, st = sample(ctx, to_dev(a), n, ns, perm=to_dev_u32(perm))
    assert int(st.item()) == ssbh.E_INVAL


def test_streamed_equals_direct_large(ctx):
    """2^28 bits, 1024 sub-blocks, keyed: the two gathers agree in full."""
    import torch
    n, ns = 1 << 28, 1024
    d_a = to_dev(uniform_bits(n, 267))
    perm = ctx.permutation(0x2828, n)
    s0, _, _, st0 = sample(ctx, d_a, n, ns, perm=perm)
    s1, _, _, st1 = sample(ctx, d_a, n, ns, perm=perm, path=1)
    assert int(st0.item()) == 0 and int(st1.item()) == 0
    assert torch.equal(s0[: n // 64], s1[: n // 64])


def test_one_overfilled_chunk_falls_back(ctx, orc):
    """A permutation that is random except for its first chunk, which maps
    into the first window only: that one cell overflows, the whole gather
    falls back to the direct one, and the output is still the oracle's."""
    n, ns = 1 << 26, 32
    a = uniform_bits(n, 268)
    rng = np.random.default_rng(269)
    head = 1 << 18
    perm = np.concatenate([rng.permutation(head),
                           head + rng.permutation(n - head)]).astype(np.uint32)
    sub, _, _, st = sample(ctx, to_dev(a), n, ns, perm=to_dev_u32(perm))
    assert int(st.item()) == 0
    osub, _, _, _ = orc.sample(a, n, ns, orc.SAMPLE_PERMUTE, assign=perm)
    got = to_host(sub)[: osub.size]
    assert np.array_equal(got, osub), first_diff(got, osub)


def test_keyed_gather_keeps_its_bucketing(ctx, orc):
    """The streaming gather of the context's keyed permutation keeps its
    bucketing for the next call with the same key and split: a second call
    on new input bits, another key, an aborting call (whose bucket pass does
    nothing, so nothing may be kept) and the first key again all give the
    oracle's sub-blocks."""
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns = 1 << 26, 64
    perms = {k: orc.permutation(n, k) for k in (0x71, 0x72)}
    for key, seed, l_ub in [(0x71, 1, 0), (0x71, 2, 0), (0x72, 3, 0),
                            (0x71, 4, 1000), (0x71, 5, 0)]:
        a = uniform_bits(n, 280 + seed)
        sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, ssbh.SAMPLE_PERMUTE,
                                     key=key, l_ub=l_ub)
        torch.cuda.synchronize()
        if l_ub:
            assert int(st.item()) == ssbh.E_ABORT_OVERSIZE
            continue
        assert int(st.item()) == 0
        osub, _, _, _ = orc.sample(a, n, ns, orc.SAMPLE_PERMUTE,
                                   assign=perms[key])
        got = to_host(sub)[: osub.size]
        assert np.array_equal(got, osub), (key, seed, first_diff(got, osub))
