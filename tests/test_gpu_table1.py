"""GPU: the input/output sizes of the paper's FPGA experiment (Table I),
hashed by the FFT hash as one block ("traditional") and by the sub-block
method (i.i.d. division into 20 sub-blocks, each with its own seed),
against the oracle on sampled output rows and, at the smallest size, against
the bit-sliced kernel on every bit."""

import numpy as np
import pytest

from tests.gpu_util import to_dev, to_host
from workloads import table1_instance, uniform_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02856_amd import ssbh
    c = ssbh.Context(0)
    yield c
    c.close()


def bit(words, k):
    return (int(words[k >> 6]) >> (k & 63)) & 1


def traditional(ctx, c, kernel):
    import torch
    from paper_2308_02856_amd import ssbh
    n, m = c["n_bits"], c["m_bits"]
    x = uniform_bits(n, c["input_seed"])
    seed = uniform_bits(n + m - 1, c["seed_seed"])
    ln = torch.tensor([n], dtype=torch.int64, device="cuda")
    wo = torch.zeros(1, dtype=torch.int64, device="cuda")
    out, tot, st = ctx.hash_batch(to_dev(x), x.size, ln, wo, 1, to_dev(seed),
                                  n + m - 1, m, out_rule=ssbh.OUT_FIXED, out_a=m,
                                  kernel=kernel)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(tot.item()) == m
    return x, seed, to_host(out)


def sub_block_method(ctx, c, kernel):
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns, lt = c["n_bits"], c["n_sub"], c["sub_out"]
    x = uniform_bits(n, c["input_seed"])
    l_ub, _ = ssbh.ub_threshold(n, 1.0 / ns, ns, 1e-8)
    S = l_ub + lt - 1
    seeds = uniform_bits(ns * S, c["sub_seed_seed"])
    sub, ln, wo, st = ctx.sample(to_dev(x), n, ns, ssbh.SAMPLE_IID,
                                 key=c["sample_key"], l_ub=l_ub)
    out, tot, st2 = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, to_dev(seeds),
                                   ns * S, lt, out_rule=ssbh.OUT_FIXED, out_a=lt,
                                   seed_stride=S, kernel=kernel)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(st2.item()) == 0
    assert int(tot.item()) == ns * lt
    return x, seeds, S, l_ub, to_host(out)


def test_smallest_size_fft_equals_valu_and_oracle(ctx, orc):
    """96.04 Mbit -> 6.054 Mbit: both ways, FFT == bit-sliced kernel on every
    bit and sampled rows == the oracle."""
    from paper_2308_02856_amd import ssbh
    c = table1_instance(0)
    n, m = c["n_bits"], c["m_bits"]
    x, seed, got = traditional(ctx, c, ssbh.K_FFT)
    _, _, ref = traditional(ctx, c, ssbh.K_VALU)
    assert np.array_equal(got, ref)
    rng = np.random.default_rng(1)
    for r in [0, m - 1] + [int(v) for v in rng.integers(0, m, 4)]:
        assert bit(got, r) == orc.toeplitz_rowwin(x, n, seed, n + m - 1, 0, m, r), r
    x, seeds, S, l_ub, got = sub_block_method(ctx, c, ssbh.K_FFT)
    _, _, _, _, ref = sub_block_method(ctx, c, ssbh.K_VALU)
    assert np.array_equal(got, ref)
    ns, lt = c["n_sub"], c["sub_out"]
    osub, oln, owo, ost = orc.sample(x, n, ns, orc.SAMPLE_IID, key=c["sample_key"],
                                     l_ub=l_ub)
    assert ost == 0
    for j in [0, 7, ns - 1]:
        xj = osub[int(owo[j]):]
        for r in [0, lt - 1, int(rng.integers(0, lt))]:
            want = orc.toeplitz_rowwin(xj, int(oln[j]), seeds, ns * S, j * S, lt, r)
            assert bit(got, j * lt + r) == want, (j, r)


def test_largest_size_traditional_fft(ctx, orc):
    """1920 Mbit -> 152.56 Mbit as one block (transform length 2^31, four
    levels): sampled rows against the oracle."""
    from paper_2308_02856_amd import ssbh
    c = table1_instance(4)
    n, m = c["n_bits"], c["m_bits"]
    x, seed, got = traditional(ctx, c, ssbh.K_FFT)
    assert ctx.last_schedule().endswith(":L%d" % (1 << 31))
    rng = np.random.default_rng(5)
    for r in [0, 1, m - 1] + [int(v) for v in rng.integers(0, m, 4)]:
        assert bit(got, r) == orc.toeplitz_rowwin(x, n, seed, n + m - 1, 0, m, r), r


def test_largest_size_sub_block_method(ctx, orc):
    """1920 Mbit into 20 sub-blocks of about 96 Mbit, 7.628 Mbit out each,
    independent seeds: sampled rows of three sub-blocks against the oracle."""
    from paper_2308_02856_amd import ssbh
    c = table1_instance(4)
    n, ns, lt = c["n_bits"], c["n_sub"], c["sub_out"]
    x, seeds, S, l_ub, got = sub_block_method(ctx, c, ssbh.K_FFT)
    osub, oln, owo, ost = orc.sample(x, n, ns, orc.SAMPLE_IID, key=c["sample_key"],
                                     l_ub=l_ub)
    assert ost == 0
    rng = np.random.default_rng(6)
    for j in [0, 11, ns - 1]:
        xj = osub[int(owo[j]):]
        for r in [0, lt - 1, int(rng.integers(0, lt))]:
            want = orc.toeplitz_rowwin(xj, int(oln[j]), seeds, ns * S, j * S, lt, r)
            assert bit(got, j * lt + r) == want, (j, r)
