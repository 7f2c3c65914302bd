"""GPU: sampling with sifting flags (Sec. III.B step 2) and the abort
threshold calculator (Sec. III.D), against the oracle (bit-exact; the
threshold is the same integer on both sides, both computed in double)."""

import numpy as np
import pytest

from tests.gpu_util import first_diff, to_dev, to_dev_u32, to_host
from workloads import (assignment, bernoulli_bits, pack_bits, permutation,
                       uniform_bits)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02856_amd import ssbh
    c = ssbh.Context(0)
    yield c
    c.close()


def keep_bits(n, pk, seed):
    if pk >= 1.0:
        return pack_bits(np.ones(n, dtype=np.uint8))
    if pk <= 0.0:
        return pack_bits(np.zeros(n, dtype=np.uint8))
    return bernoulli_bits(n, pk, seed)


def check_sampled(ln, wo, sub, oln, owo, osub, ns):
    assert np.array_equal(to_host(ln)[:ns], oln)
    assert np.array_equal(to_host(wo)[:ns], owo)
    got = to_host(sub)[: osub.size]
    assert np.array_equal(got, osub), first_diff(got, osub)


@pytest.mark.parametrize("n,ns,pk", [(1, 1, 1.0), (1000, 7, 0.5),
                                     ((1 << 20) + 77, 300, 0.8),
                                     ((1 << 18) + 1, 2048, 0.3),
                                     (300000, 5000, 0.9),      # ballot path
                                     (65536, 64, 0.0), (99999, 16, 1.0)])
def test_sifted_iid_matches_oracle(ctx, orc, n, ns, pk):
    import torch
    from paper_2308_02856_amd import ssbh
    a = bernoulli_bits(n, 0.4, n % 997)
    keep = keep_bits(n, pk, n % 991)
    key = 0x51F7 + ns
    sub, ln, wo, st = ctx.sample_sifted(to_dev(a), to_dev(keep), n, ns,
                                        ssbh.SAMPLE_IID, key=key)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=key,
                                   keep=keep)
    check_sampled(ln, wo, sub, oln, owo, osub, ns)


def test_sifted_explicit_matches_oracle(ctx, orc):
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns = 123457, 11
    a = uniform_bits(n, 5)
    keep = keep_bits(n, 0.6, 6)
    v = assignment(n, ns, 7)
    sub, ln, wo, st = ctx.sample_sifted(to_dev(a), to_dev(keep), n, ns,
                                        ssbh.SAMPLE_EXPLICIT,
                                        assign=to_dev_u32(v))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_EXPLICIT, assign=v,
                                   keep=keep)
    check_sampled(ln, wo, sub, oln, owo, osub, ns)


def test_sifted_rejects_permutation_and_null_flags(ctx):
    from paper_2308_02856_amd import ssbh
    n, ns = 4096, 4
    a = to_dev(uniform_bits(n, 1))
    keep = to_dev(keep_bits(n, 0.5, 2))
    perm = to_dev_u32(permutation(n, 3))
    with pytest.raises(ssbh.SsbhError) as e:
        ctx.sample_sifted(a, keep, n, ns, ssbh.SAMPLE_PERMUTE, assign=perm)
    assert e.value.status == ssbh.E_INVAL
    with pytest.raises(ssbh.SsbhError):
        ctx.sample_sifted(a, None, n, ns, ssbh.SAMPLE_IID, key=1)


def test_abort_counts_kept_bits_only(ctx, orc):
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns = 200000, 20
    a = uniform_bits(n, 8)
    keep = keep_bits(n, 0.5, 9)
    key = 0xAB
    _, oln, _, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=key, keep=keep)
    top = int(oln.max())
    for l_ub, want in ((top, 0), (top - 1, ssbh.E_ABORT_OVERSIZE)):
        _, _, _, st = ctx.sample_sifted(to_dev(a), to_dev(keep), n, ns,
                                        ssbh.SAMPLE_IID, key=key, l_ub=l_ub)
        torch.cuda.synchronize()
        assert int(st.item()) == want, l_ub


def test_sifted_then_hash_matches_oracle(ctx, orc):
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns = (1 << 21) + 3, 96
    a = bernoulli_bits(n, 0.3, 10)
    keep = keep_bits(n, 0.7, 11)
    key = 0x5EED
    sub, ln, wo, st = ctx.sample_sifted(to_dev(a), to_dev(keep), n, ns,
                                        ssbh.SAMPLE_IID, key=key)
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=key,
                                   keep=keep)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 2, 5)
    cap = int(om.max())
    seed_bits = int(oln.max()) + cap - 1
    seed = uniform_bits(seed_bits, 12)
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed, seed_bits, 0, cap)
    for kern in (ssbh.K_VALU, ssbh.K_MFMA_I8):
        out, tot, st2 = ctx.hash_batch(sub, sub.numel(), ln, wo, ns,
                                       to_dev(seed), seed_bits, cap,
                                       out_rule=ssbh.OUT_RATIO, out_a=2,
                                       out_b=5, kernel=kern, status=st,
                                       reset_status=False)
        torch.cuda.synchronize()
        assert int(st2.item()) == 0 and int(tot.item()) == wtot
        assert np.array_equal(to_host(out)[: want.size], want), kern


def test_sifted_graph_pipeline_replays(ctx, orc):
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns, m = 500000, 40, 3000
    a = uniform_bits(n, 13)
    keep = keep_bits(n, 0.75, 14)
    key = 0x77
    d_in, d_keep = to_dev(a), to_dev(keep)
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=key,
                                   keep=keep)
    seed_bits = int(oln.max()) + m - 1 + 1000
    seed = uniform_bits(seed_bits, 15)
    want, wtot = orc.hash_batch(osub, oln, owo, np.full(ns, m, np.uint64),
                                seed, seed_bits, 0, m)
    cap = (n + 63) // 64 + ns
    sub = torch.empty(cap, dtype=torch.int64, device="cuda")
    ln = torch.empty(ns, dtype=torch.int64, device="cuda")
    wo = torch.empty(ns, dtype=torch.int64, device="cuda")
    out = torch.empty((ns * m + 63) // 64, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pipe = ctx.pipeline(d_in=d_in, d_keep=d_keep, n_bits=n, n_sub=ns,
                        mode=ssbh.SAMPLE_IID, sample_key=key, d_sub=sub,
                        sub_capacity_words=cap, d_len=ln, d_word_off=wo,
                        out_rule=ssbh.OUT_FIXED, out_a=m, out_b=1,
                        d_seed=to_dev(seed), seed_bits=seed_bits, m_cap=m,
                        kernel=ssbh.K_VALU, d_out=out,
                        out_capacity_bits=ns * m, d_out_total_bits=tot,
                        d_status=st)
    for _ in range(3):
        out.fill_(-1)
        torch.cuda.synchronize()
        pipe.launch()
        torch.cuda.synchronize()
        assert int(st.item()) == 0 and int(tot.item()) == wtot
        assert np.array_equal(to_host(out)[: want.size], want)
    pipe.close()


@pytest.mark.parametrize("n,p,ns,eps", [(2 ** 28, 1 / 2048, 2048, 1e-8),
                                        (2 ** 28, 0.3 / 2048, 2048, 1e-8),
                                        (2 ** 24, 0.3 / 128, 128, 1e-6),
                                        (10 ** 5, 0.05, 20, 1e-10),
                                        (200, 0.5, 2, 1e-30),
                                        (2 ** 31, 0.9 / 20, 20, 1e-9),
                                        (1000, 0.001, 1, 0.5)])
def test_ub_threshold_matches_oracle(orc, n, p, ns, eps):
    from paper_2308_02856_amd import ssbh
    L, at = ssbh.ub_threshold(n, p, ns, eps)
    assert L == orc.ub_threshold(n, p, ns, eps)
    assert at == pytest.approx(ns * orc.ub_tail(n, p, L), rel=1e-9, abs=1e-300)
    assert at <= eps


def test_ub_threshold_rejects_bad_arguments():
    from paper_2308_02856_amd import ssbh
    for args in ((100, 0.0, 2, 1e-3), (100, 1.0, 2, 1e-3), (100, 0.5, 0, 1e-3),
                 (100, 0.5, 2, 0.0), (0, 0.5, 2, 1e-3)):
        with pytest.raises(ssbh.SsbhError):
            ssbh.ub_threshold(*args)
