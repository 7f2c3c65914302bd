"""GPU: both scatter kernels of the i.i.d. / explicit sampling (a workgroup
of four wavefronts per segment, and one wavefront per segment) give the
oracle's sub-blocks bit for bit, with and without sifting flags."""

import numpy as np
import pytest

from tests.gpu_util import first_diff, to_dev, to_dev_u32, to_host
from workloads import assignment, bernoulli_bits

pytestmark = pytest.mark.gpu

CASES = [  # (n, n_sub, keep probability or None)
    (1, 1, None), (63, 2, None), (1000, 7, None), ((1 << 20) + 77, 300, None),
    ((1 << 18) + 1, 2048, 0.5), ((1 << 21) + 5, 2048, None), (200000, 256, 0.9),
    (150000, 257, None), (99999, 1000, 0.3), (4096 * 3 + 17, 3, 1.0),
    (50000, 1500, 0.0), ((1 << 21) + 3, 4096, None), (300000, 3000, 0.6),
]
PATHS = [0, 1]


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02856_amd import ssbh
    c = ssbh.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n,ns,pk", CASES)
def test_iid_paths_match_oracle(ctx, orc, path, n, ns, pk):
    import torch
    from paper_2308_02856_amd import ssbh
    a = bernoulli_bits(n, 0.45, n % 1013)
    key = 0xC0FFEE + ns
    keep = None
    if pk is not None:
        keep = (bernoulli_bits(n, pk, n % 1019) if 0.0 < pk < 1.0 else
                np.full((n + 63) // 64, np.uint64(0 if pk == 0.0 else ~np.uint64(0)),
                        dtype=np.uint64))
        if pk == 1.0 and n % 64:
            keep[-1] &= np.uint64((1 << (n % 64)) - 1)
    ctx.set_sample_path(path)
    try:
        if keep is None:
            sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, ssbh.SAMPLE_IID, key=key)
        else:
            sub, ln, wo, st = ctx.sample_sifted(to_dev(a), to_dev(keep), n, ns,
                                                ssbh.SAMPLE_IID, key=key)
        torch.cuda.synchronize()
    finally:
        ctx.set_sample_path(0)
    assert int(st.item()) == 0
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=key, keep=keep)
    assert np.array_equal(to_host(ln)[:ns], oln)
    assert np.array_equal(to_host(wo)[:ns], owo)
    got = to_host(sub)[: osub.size]
    assert np.array_equal(got, osub), first_diff(got, osub)


@pytest.mark.parametrize("path", PATHS)
def test_explicit_paths_match_oracle(ctx, orc, path):
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns = (1 << 19) + 11, 700
    a = bernoulli_bits(n, 0.5, 5)
    v = assignment(n, ns, 6)
    ctx.set_sample_path(path)
    try:
        sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, ssbh.SAMPLE_EXPLICIT,
                                     assign=to_dev_u32(v))
        torch.cuda.synchronize()
    finally:
        ctx.set_sample_path(0)
    assert int(st.item()) == 0
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_EXPLICIT, assign=v)
    assert np.array_equal(to_host(ln)[:ns], oln)
    got = to_host(sub)[: osub.size]
    assert np.array_equal(got, osub), first_diff(got, osub)


@pytest.mark.parametrize("path", PATHS)
def test_explicit_concentrated_assignment(ctx, orc, path):
    """Every round of whole segments in one sub-block (the largest per-quarter
    counts the scatter sees), the rest spread over a few sub-blocks."""
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns = (1 << 20) + 333, 2048
    a = bernoulli_bits(n, 0.5, 9)
    v = np.zeros(n, dtype=np.uint32)
    v[n // 2:] = (np.arange(n - n // 2) % 3 + 2045).astype(np.uint32)
    ctx.set_sample_path(path)
    try:
        sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, ssbh.SAMPLE_EXPLICIT,
                                     assign=to_dev_u32(v))
        torch.cuda.synchronize()
    finally:
        ctx.set_sample_path(0)
    assert int(st.item()) == 0
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_EXPLICIT, assign=v)
    assert np.array_equal(to_host(ln)[:ns], oln)
    got = to_host(sub)[: osub.size]
    assert np.array_equal(got, osub), first_diff(got, osub)


def test_rejects_n_bits_above_limit(ctx):
    """n_bits past 2^32 - 2^20 (32-bit round indices) is refused on the host,
    before any launch."""
    from paper_2308_02856_amd import ssbh
    a = to_dev(np.zeros(4, dtype=np.uint64))
    with pytest.raises(ssbh.SsbhError) as e:
        ctx.sample(a, (1 << 32) - (1 << 20) + 1, 16, ssbh.SAMPLE_IID, key=1,
                   sub_capacity=8)
    assert e.value.status == ssbh.E_UNSUPPORTED
