"""GPU: the keyed permutation of the permutation-split sampling mode.

The library computes Durstenfeld's shuffle by parallel passes (group counts,
a scan, sorted groups and chain ends); the oracle runs the sequential loop.
They must agree entry for entry for every size and key.  Sampling in
permutation mode without a caller permutation must give the oracle's
permute-split of the oracle's permutation.
"""

import numpy as np
import pytest

from tests.gpu_util import first_diff, to_dev, to_host
from workloads import uniform_bits

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 5, 64, 4095, 4096, 4097, 65537, (1 << 20) + 17]
KEYS = [0, 1, 0x2308028560000101, 2**64 - 1]


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02856_amd import ssbh
    c = ssbh.Context(0)
    yield c
    c.close()


def perm_host(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("key", KEYS)
def test_permutation_matches_oracle(ctx, orc, n, key):
    import torch
    got = ctx.permutation(key, n)
    torch.cuda.synchronize()
    want = orc.permutation(n, key)
    assert np.array_equal(perm_host(got)[:n], want), (n, key)


def test_permutation_large(ctx, orc):
    """2^24 + 3 entries (three scan levels of block sums are not needed here,
    two are): equal to the oracle and a permutation."""
    import torch
    n, key = (1 << 24) + 3, 0xABCDEF12345
    got = perm_host(ctx.permutation(key, n))[:n]
    torch.cuda.synchronize()
    assert np.array_equal(np.bincount(got, minlength=n), np.ones(n, np.int64))
    assert np.array_equal(got, orc.permutation(n, key))


def test_permutation_many_keys_small_n(ctx, orc):
    """n = 5 over 400 keys: every result equals the oracle's (whose
    uniformity over the 120 permutations is pinned on the CPU)."""
    import torch
    seen = set()
    for k in range(400):
        key = 0x5151 + 7919 * k
        got = tuple(perm_host(ctx.permutation(key, 5))[:5].tolist())
        torch.cuda.synchronize()
        assert got == tuple(orc.permutation(5, key).tolist()), key
        seen.add(got)
    assert len(seen) > 100


def test_permutation_zero_length_is_a_no_op(ctx):
    import torch
    out = torch.full((4,), 7, dtype=torch.int32, device="cuda")
    ctx.permutation(99, 0, out=out)
    torch.cuda.synchronize()
    assert out.tolist() == [7, 7, 7, 7]


@pytest.mark.parametrize("n,ns", [(1 << 20, 16), (96 * 1000, 96), (7, 7)])
def test_keyed_permute_split_matches_oracle(ctx, orc, n, ns):
    """ssbh_sample in permutation mode with d_assign = NULL builds the keyed
    permutation of sample_key itself."""
    import torch
    from paper_2308_02856_amd import ssbh
    key = 0x77 + n
    a = uniform_bits(n, n % 997)
    sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, ssbh.SAMPLE_PERMUTE,
                                 key=key)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_PERMUTE,
                                   assign=orc.permutation(n, key))
    got = to_host(sub)[: osub.size]
    assert np.array_equal(got, osub), first_diff(got, osub)
    assert np.array_equal(to_host(ln)[:ns], oln)
    assert np.array_equal(to_host(wo)[:ns], owo)


def test_keyed_split_reuses_and_rebuilds_its_permutation(ctx, orc):
    """The context keeps the keyed permutation of the last (key, n): the
    same key twice, then another key, then another length, each equal to
    the oracle's split of the oracle's permutation."""
    import torch
    from paper_2308_02856_amd import ssbh
    for n, ns, key in [(1 << 16, 8, 0x11), (1 << 16, 8, 0x11), (1 << 16, 8, 0x12),
                       ((1 << 16) + 8, 8, 0x12), (1 << 16, 8, 0x11)]:
        a = uniform_bits(n, 70 + n % 7 + key)
        sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, ssbh.SAMPLE_PERMUTE,
                                     key=key)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        osub, _, _, _ = orc.sample(a, n, ns, orc.SAMPLE_PERMUTE,
                                   assign=orc.permutation(n, key))
        got = to_host(sub)[: osub.size]
        assert np.array_equal(got, osub), (n, key, first_diff(got, osub))
