"""GPU: the captured graph pipeline and the autotuner.

Graph replays are checked against eager results after every replay, with
eager work (input changes, synchronisations) between the replays.  The
autotuner must leave a valid result and a table entry, and AUTO calls after
tuning must give the same bits as the oracle.
"""

import numpy as np
import pytest

from tests.gpu_util import first_diff, to_dev, to_dev_u32, to_host
from workloads import bernoulli_bits, config, uniform_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02856_amd import ssbh
    c = ssbh.Context(0)
    yield c
    c.close()


def test_graph_replays_match_eager(ctx, orc):
    import torch
    from paper_2308_02856_amd import ssbh
    c = config("small")
    n, ns, L, m = c["n_bits"], c["n_sub"], c["sub_bits"], c["out_a"]
    stride = L + m - 1
    seed_bits = ns * stride
    perm = orc.permutation(n, c["perm_key"])
    seed = to_dev(uniform_bits(seed_bits, c["seed_seed"]))
    d_in = to_dev(uniform_bits(n, c["input_seed"]))
    d_perm = to_dev_u32(perm)
    sub_cap = ns * ((L + 63) // 64)
    sub = torch.empty(sub_cap, dtype=torch.int64, device="cuda")
    ln = torch.empty(ns, dtype=torch.int64, device="cuda")
    wo = torch.empty(ns, dtype=torch.int64, device="cuda")
    out = torch.empty(ns * m // 64, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pipe = ctx.pipeline(d_in=d_in, n_bits=n, n_sub=ns,
                        mode=ssbh.SAMPLE_PERMUTE, d_assign=d_perm,
                        d_sub=sub, sub_capacity_words=sub_cap, d_len=ln,
                        d_word_off=wo, out_rule=ssbh.OUT_FIXED, out_a=m,
                        out_b=1, d_seed=seed, seed_bits=seed_bits,
                        seed_stride=stride, m_cap=m, kernel=ssbh.K_VALU,
                        d_out=out, out_capacity_bits=ns * m,
                        d_out_total_bits=tot, d_status=st)
    for rep in range(5):
        a = uniform_bits(n, 500 + rep)
        d_in.copy_(to_dev(a))              # eager work between replays
        pipe.launch()
        torch.cuda.synchronize()
        got = to_host(out).copy()
        assert int(st.item()) == 0
        e_sub, e_ln, e_wo, e_st = ctx.sample(d_in, n, ns, ssbh.SAMPLE_PERMUTE,
                                             assign=d_perm)
        e_out, e_tot, _ = ctx.hash_batch(e_sub, e_sub.numel(), e_ln, e_wo, ns,
                                         seed, seed_bits, m,
                                         out_rule=ssbh.OUT_FIXED, out_a=m,
                                         seed_stride=stride, status=e_st,
                                         reset_status=False)
        torch.cuda.synchronize()
        assert np.array_equal(got, to_host(e_out)), (rep, first_diff(got, to_host(e_out)))
        if rep == 0:
            osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_PERMUTE,
                                           assign=perm)
            want, _ = orc.hash_batch(osub, oln, owo, np.full(ns, m, np.uint64),
                                     to_host(seed), seed_bits, stride, m)
            assert np.array_equal(got[: want.size], want)
    pipe.close()


def test_graph_iid_hash_only_and_mfma(ctx, orc):
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns = (1 << 20) + 5, 128
    a = bernoulli_bits(n, 0.3, 61)
    d_in = to_dev(a)
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=62)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 2, 5)
    cap = int(om.max())
    seed_bits = int(oln.max()) + cap - 1
    seed_h = uniform_bits(seed_bits, 63)
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed_h, seed_bits, 0, cap)
    seed = to_dev(seed_h)
    sub_cap = (n + 63) // 64 + ns
    sub = torch.empty(sub_cap, dtype=torch.int64, device="cuda")
    ln = torch.empty(ns, dtype=torch.int64, device="cuda")
    wo = torch.empty(ns, dtype=torch.int64, device="cuda")
    out = torch.empty((wtot + 63) // 64, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pipe = ctx.pipeline(d_in=d_in, n_bits=n, n_sub=ns, mode=ssbh.SAMPLE_IID,
                        sample_key=62, d_sub=sub, sub_capacity_words=sub_cap,
                        d_len=ln, d_word_off=wo, out_rule=ssbh.OUT_RATIO,
                        out_a=2, out_b=5, d_seed=seed, seed_bits=seed_bits,
                        m_cap=cap, kernel=ssbh.K_MFMA_I8, d_out=out,
                        out_capacity_bits=wtot, d_out_total_bits=tot,
                        d_status=st)
    for _ in range(4):
        out.fill_(-1)
        pipe.launch()
        torch.cuda.synchronize()
        assert int(st.item()) == 0 and int(tot.item()) == wtot
        assert np.array_equal(to_host(out)[: want.size], want)
    pipe.close()


def test_autotune_then_auto_is_exact(ctx, orc):
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns = (1 << 21) + 77, 96
    a = bernoulli_bits(n, 0.4, 71)
    sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, ssbh.SAMPLE_IID, key=72)
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=72)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 2, 5)
    cap = int(om.max())
    seed_bits = int(oln.max()) + cap - 1
    seed_h = uniform_bits(seed_bits, 73)
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed_h, seed_bits, 0, cap)
    report = ctx.tune(sub, sub.numel(), ln, wo, ns, to_dev(seed_h), seed_bits,
                      cap, out_rule=ssbh.OUT_RATIO, out_a=2, out_b=5,
                      status=st)
    assert "mfma" in report and "valu" in report
    table = ctx.tune_table()
    assert table.startswith("shared/")
    out, tot, st2 = ctx.hash_batch(sub, sub.numel(), ln, wo, ns,
                                   to_dev(seed_h), seed_bits, cap,
                                   out_rule=ssbh.OUT_RATIO, out_a=2, out_b=5,
                                   kernel=ssbh.K_AUTO)
    torch.cuda.synchronize()
    assert int(st2.item()) == 0 and int(tot.item()) == wtot
    assert np.array_equal(to_host(out)[: want.size], want)


FUSED_CASES = [  # (n_sub, L, out rule, a, b, independent seeds)
    (8, 1 << 15, 0, 1 << 14, 1, True),      # the small workload's shape
    (8, 1 << 15, 0, 1 << 14, 1, False),
    (5, 1000, 0, 320, 1, False),            # partial last row tile
    (3, 1 << 16, 0, 192, 1, True),          # longest fused sub-block
    (1, 4097, 0, 640, 1, False),            # one sub-block, ragged length
    (16, 1600, 1, 2, 5, True),              # ratio rule: m = 640
    (7, 33, 0, 64, 1, True),                # m > n
    (5, 1 << 16, 0, 128, 1, True),          # input of 5 * 2^16 bits
    (2, 1 << 16, 0, 40960, 1, False),       # 80 row tiles a sub-block
]


@pytest.mark.parametrize("ns,L,rule,a,b,indep", FUSED_CASES)
def test_fused_small_pipeline_matches_oracle(ctx, orc, ns, L, rule, a, b, indep):
    """Small permutation-split jobs with equal sub-blocks and 64-bit aligned
    outputs replay as two fused kernels: every replay gives the oracle's
    sub-blocks, lengths, offsets and output, equal to the eager calls."""
    import torch
    from paper_2308_02856_amd import ssbh
    n = ns * L
    m = a if rule == 0 else L * a // b
    stride = L + m - 1 if indep else 0
    seed_bits = (ns - 1) * stride + L + m - 1
    perm = orc.permutation(n, 0x3300 + n)
    d_perm = to_dev_u32(perm)
    seed_h = uniform_bits(seed_bits, n + 1)
    seed = to_dev(seed_h)
    wl = (L + 63) // 64
    sub_cap = ns * wl
    d_in = to_dev(uniform_bits(n, n))
    sub = torch.empty(sub_cap, dtype=torch.int64, device="cuda")
    ln = torch.empty(ns, dtype=torch.int64, device="cuda")
    wo = torch.empty(ns, dtype=torch.int64, device="cuda")
    out = torch.empty(ns * m // 64, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pipe = ctx.pipeline(d_in=d_in, n_bits=n, n_sub=ns,
                        mode=ssbh.SAMPLE_PERMUTE, d_assign=d_perm,
                        d_sub=sub, sub_capacity_words=sub_cap, d_len=ln,
                        d_word_off=wo, out_rule=rule, out_a=a, out_b=b,
                        d_seed=seed, seed_bits=seed_bits, seed_stride=stride,
                        m_cap=m, kernel=ssbh.K_VALU, d_out=out,
                        out_capacity_bits=ns * m, d_out_total_bits=tot,
                        d_status=st)
    for rep in range(3):
        x = uniform_bits(n, 900 + rep)
        d_in.copy_(to_dev(x))
        out.fill_(-1)
        st.fill_(7)
        pipe.launch()
        torch.cuda.synchronize()
        assert int(st.item()) == 0 and int(tot.item()) == ns * m
        osub, oln, owo, _ = orc.sample(x, n, ns, orc.SAMPLE_PERMUTE,
                                       assign=perm)
        want, wtot = orc.hash_batch(osub, oln, owo, np.full(ns, m, np.uint64),
                                    seed_h, seed_bits, stride, m)
        assert wtot == ns * m
        got = to_host(out)
        assert np.array_equal(got, want), (rep, first_diff(got, want))
        assert np.array_equal(to_host(sub)[: osub.size], osub)
        assert np.array_equal(to_host(ln)[:ns], oln)
        assert np.array_equal(to_host(wo)[:ns], owo)
    pipe.close()


def test_fused_small_pipeline_bad_permutation(ctx):
    """An entry of pi outside [0, n) sets SSBH_E_INVAL and leaves the output
    untouched, as in the general path."""
    import torch
    from paper_2308_02856_amd import ssbh
    ns, L, m = 4, 2048, 512
    n = ns * L
    perm = np.arange(n, dtype=np.uint32)
    d_perm = to_dev_u32(perm)
    seed_bits = L + m - 1
    seed = to_dev(uniform_bits(seed_bits, 5))
    d_in = to_dev(uniform_bits(n, 6))
    sub = torch.empty(ns * L // 64, dtype=torch.int64, device="cuda")
    ln = torch.empty(ns, dtype=torch.int64, device="cuda")
    wo = torch.empty(ns, dtype=torch.int64, device="cuda")
    out = torch.empty(ns * m // 64, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pipe = ctx.pipeline(d_in=d_in, n_bits=n, n_sub=ns,
                        mode=ssbh.SAMPLE_PERMUTE, d_assign=d_perm, d_sub=sub,
                        sub_capacity_words=sub.numel(), d_len=ln,
                        d_word_off=wo, out_rule=ssbh.OUT_FIXED, out_a=m,
                        out_b=1, d_seed=seed, seed_bits=seed_bits,
                        m_cap=m, kernel=ssbh.K_AUTO, d_out=out,
                        out_capacity_bits=ns * m, d_out_total_bits=tot,
                        d_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    perm[777] = n + 5
    d_perm.copy_(to_dev_u32(perm))
    out.fill_(0x1234)
    pipe.launch()
    torch.cuda.synchronize()
    assert int(st.item()) == ssbh.E_INVAL
    assert bool((out == 0x1234).all())
    perm[777] = 777
    d_perm.copy_(to_dev_u32(perm))
    pipe.launch()
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    pipe.close()
