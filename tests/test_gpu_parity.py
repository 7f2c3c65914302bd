"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

All arithmetic is GF(2), so the bar is bit-exact equality of every compared
word or bit.  Small and medium cases are compared in full; the full-size
workloads are compared on the whole sampling output and on sampled output
rows that the oracle computes one by one.
"""

import numpy as np
import pytest

from tests.gpu_util import bit, first_diff, to_dev, to_dev_u32, to_host
from workloads import (assignment, bernoulli_bits, config, permutation,
                       uniform_bits)

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


def gpu_hash_one(ctx, S, x, n, seed, seed_bits, m, **kw):
    """One block hashed on the GPU (n_sub = 1, word offset 0)."""
    import torch
    xs = to_dev(x)
    ln = torch.tensor([n], dtype=torch.int64, device="cuda")
    wo = torch.zeros(1, dtype=torch.int64, device="cuda")
    out, tot, st = ctx.hash_batch(xs, xs.numel(), ln, wo, 1, to_dev(seed),
                                  seed_bits, m, out_rule=S.OUT_FIXED, out_a=m,
                                  out_capacity_bits=max(m, 1), **kw)
    torch.cuda.synchronize()
    assert int(st.item()) == 0, S.status_name(int(st.item()))
    assert int(tot.item()) == m
    return to_host(out)[: (m + 63) // 64]


# ------------------------------------------------------------- one block ---

SHAPES = [(1, 1), (31, 33), (64, 64), (100, 37), (1000, 1500), (4097, 2049),
          (32768 + 45, 16384 + 13), (70001, 5000), (300, 9000)]


@pytest.mark.parametrize("n,m", SHAPES)
def test_single_block_matches_oracle(ctx, S, orc, n, m):
    x = uniform_bits(n, n + 3 * m)
    seed = uniform_bits(n + m - 1, 7 * n + m)
    want = orc.toeplitz(x, n, seed, n + m - 1, m)
    got = gpu_hash_one(ctx, S, x, n, seed, n + m - 1, m)
    assert np.array_equal(got, want), first_diff(got, want)


SCHEDULES = [(8, 4, 0), (16, 4, 0), (32, 4, 0), (16, 2, 0), (32, 2, 0),
             (16, 8, 0), (16, 4, 256), (32, 2, 512), (8, 4, 1024)]


@pytest.mark.parametrize("r,w,tc", SCHEDULES)
def test_every_schedule_is_bit_identical(ctx, S, orc, r, w, tc):
    n, m = 50000 + 17, 20000 + 5
    x = bernoulli_bits(n, 0.3, 11)
    seed = uniform_bits(n + m - 1, 12)
    want = orc.toeplitz(x, n, seed, n + m - 1, m)
    ctx.set_schedule(r, w, tc)
    try:
        got = gpu_hash_one(ctx, S, x, n, seed, n + m - 1, m, kernel=S.K_VALU)
    finally:
        ctx.set_schedule(0, 0, 0)
    assert np.array_equal(got, want), first_diff(got, want)


def test_input_bits_past_n_are_ignored(ctx, S, orc):
    n, m = 1000, 700
    x = uniform_bits(n, 21)
    dirty = x.copy()
    dirty[-1] |= np.uint64(0xFFFFFF0000000000)
    seed = uniform_bits(n + m - 1, 22)
    want = orc.toeplitz(x, n, seed, n + m - 1, m)
    assert np.array_equal(gpu_hash_one(ctx, S, dirty, n, seed, n + m - 1, m),
                          want)


# -------------------------------------------------------------- sampling ---

@pytest.mark.parametrize("n,ns", [(1, 1), (1000, 7), (65536, 1), (100003, 64),
                                  (1 << 20, 2048), (300000, 16384),
                                  (777777, 3)])
def test_sample_iid_matches_oracle(ctx, S, orc, n, ns):
    import torch
    a = bernoulli_bits(n, 0.3, n ^ ns)
    key = 0x5EED0000 + ns
    sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, S.SAMPLE_IID, key=key)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=key)
    assert np.array_equal(to_host(ln)[:ns], oln)
    assert np.array_equal(to_host(wo)[:ns], owo)
    got = to_host(sub)[: osub.size]
    assert np.array_equal(got, osub), first_diff(got, osub)


def test_sample_explicit_matches_oracle(ctx, S, orc):
    import torch
    n, ns = 123457, 300
    a = uniform_bits(n, 5)
    v = assignment(n, ns, 6)
    v[v == 17] = 18            # one empty sub-block
    sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, S.SAMPLE_EXPLICIT,
                                 assign=to_dev_u32(v))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_EXPLICIT, assign=v)
    assert int(oln[17]) == 0
    assert np.array_equal(to_host(ln)[:ns], oln)
    assert np.array_equal(to_host(sub)[: osub.size], osub)


def test_sample_explicit_rejects_out_of_range(ctx, S):
    import torch
    n, ns = 5000, 10
    v = assignment(n, ns, 1)
    v[1234] = ns
    _, _, _, st = ctx.sample(to_dev(uniform_bits(n, 1)), n, ns,
                             S.SAMPLE_EXPLICIT, assign=to_dev_u32(v))
    torch.cuda.synchronize()
    assert int(st.item()) == S.E_INVAL


@pytest.mark.parametrize("n,ns", [(1 << 12, 8), (960, 3), (64 * 5, 5),
                                  (1 << 18, 8)])
def test_sample_permute_matches_oracle(ctx, S, orc, n, ns):
    import torch
    a = uniform_bits(n, 31)
    perm = permutation(n, 32)
    sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, S.SAMPLE_PERMUTE,
                                 assign=to_dev_u32(perm))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_PERMUTE, assign=perm)
    assert np.array_equal(to_host(ln)[:ns], oln)
    assert np.array_equal(to_host(wo)[:ns], owo)
    assert np.array_equal(to_host(sub)[: osub.size], osub)


def test_abort_rule_and_untouched_output(ctx, S, orc):
    import torch
    n, ns = 200000, 16
    a = uniform_bits(n, 41)
    _, oln, _, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=42)
    mx = int(oln.max())
    sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, S.SAMPLE_IID, key=42,
                                 l_ub=mx - 1)
    torch.cuda.synchronize()
    assert int(st.item()) == S.E_ABORT_OVERSIZE
    seed = to_dev(uniform_bits(mx + 1000, 43))
    out = torch.full((100,), 0x1234, dtype=torch.int64, device="cuda")
    out, tot, st2 = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed,
                                   mx + 1000, 1000, out_rule=S.OUT_FIXED,
                                   out_a=1000, out=out,
                                   out_capacity_bits=6400, status=st,
                                   reset_status=False)
    torch.cuda.synchronize()
    assert int(st2.item()) == S.E_ABORT_OVERSIZE
    assert bool((out == 0x1234).all())
    _, _, _, st = ctx.sample(to_dev(a), n, ns, S.SAMPLE_IID, key=42, l_ub=mx)
    torch.cuda.synchronize()
    assert int(st.item()) == 0


# ------------------------------------------------------ batch end to end ---

@pytest.mark.parametrize("stride_mode", ["shared", "independent"])
def test_sample_and_hash_batch_matches_oracle(ctx, S, orc, stride_mode):
    import torch
    n, ns = (1 << 20) + 12345, 96
    a = bernoulli_bits(n, 0.3, 51)
    key = 0xABCDEF
    sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, S.SAMPLE_IID, key=key)
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=key)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 2, 5)
    cap = int(om.max())
    nmax = int(oln.max())
    stride = 0 if stride_mode == "shared" else nmax + cap - 1
    seed_bits = (ns - 1) * stride + nmax + cap - 1
    seed = uniform_bits(seed_bits, 52)
    out, tot, st = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, to_dev(seed),
                                  seed_bits, cap, out_rule=S.OUT_RATIO,
                                  out_a=2, out_b=5, seed_stride=stride,
                                  status=st, reset_status=False)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed, seed_bits, stride,
                                cap)
    assert int(tot.item()) == wtot
    got = to_host(out)[: want.size]
    assert np.array_equal(got, want), first_diff(got, want)


def test_empty_and_degenerate_sub_blocks(ctx, S, orc):
    import torch
    # sub-blocks of length 0, 1, 63, 64, 65 with fixed output length 40
    lens = [0, 1, 63, 64, 65, 0, 200]
    ns = len(lens)
    words = [(L + 63) // 64 for L in lens]
    wo = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    sub = uniform_bits(64 * int(sum(words)), 61)
    for j, L in enumerate(lens):      # zero the pad bits
        if L % 64:
            sub[int(wo[j]) + words[j] - 1] &= np.uint64((1 << (L % 64)) - 1)
    m = 40
    seed_bits = max(lens) + m - 1
    seed = uniform_bits(seed_bits, 62)
    ln_d = torch.tensor(lens, dtype=torch.int64, device="cuda")
    wo_d = to_dev(wo)
    out, tot, st = ctx.hash_batch(to_dev(sub), int(sum(words)), ln_d, wo_d, ns,
                                  to_dev(seed), seed_bits, m,
                                  out_rule=S.OUT_FIXED, out_a=m)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(tot.item()) == m * ns
    want, _ = orc.hash_batch(sub, np.array(lens, np.uint64), wo,
                             np.full(ns, m, np.uint64), seed, seed_bits, 0, m)
    assert np.array_equal(to_host(out)[: want.size], want)


def test_device_side_length_errors(ctx, S):
    import torch
    n = 1000
    x = to_dev(uniform_bits(n, 71))
    ln = torch.tensor([n], dtype=torch.int64, device="cuda")
    wo = torch.zeros(1, dtype=torch.int64, device="cuda")
    seed = to_dev(uniform_bits(n + 99, 72))
    sentinel = torch.full((4,), 77, dtype=torch.int64, device="cuda")
    # seed one bit too short
    out, _, st = ctx.hash_batch(x, x.numel(), ln, wo, 1, seed, n + 98, 100,
                                out_rule=S.OUT_FIXED, out_a=100,
                                out=sentinel.clone(), out_capacity_bits=256)
    torch.cuda.synchronize()
    assert int(st.item()) == S.E_INVAL and bool((out == 77).all())
    # output capacity too small
    out, _, st = ctx.hash_batch(x, x.numel(), ln, wo, 1, seed, n + 99, 100,
                                out_rule=S.OUT_FIXED, out_a=100,
                                out=sentinel.clone(), out_capacity_bits=99)
    torch.cuda.synchronize()
    assert int(st.item()) == S.E_INVAL and bool((out == 77).all())
    # m above the cap
    with pytest.raises(S.SsbhError):
        ctx.hash_batch(x, x.numel(), ln, wo, 1, seed, n + 99, 0,
                       out_rule=S.OUT_FIXED, out_a=100)


def test_seed_from_key_matches_oracle(ctx, orc):
    import torch
    for bits in (1, 64, 1000, 185537):
        got = to_host(ctx.seed_from_key(0xC0FFEE + bits, bits))
        torch.cuda.synchronize()
        assert np.array_equal(got[: (bits + 63) // 64],
                              orc.seed_from_key(0xC0FFEE + bits, bits))


# ---------------------------------------------------- full-size workloads ---

def test_small_workload_in_full(ctx, S, orc):
    """2^18 bits, permutation split into 8 x 2^15, 2^14 output bits each,
    independent seeds: every output bit compared."""
    import torch
    c = config("small")
    n, ns, L, m = c["n_bits"], c["n_sub"], c["sub_bits"], c["out_a"]
    a = uniform_bits(n, c["input_seed"])
    perm = orc.permutation(n, c["perm_key"])
    stride = L + m - 1
    seed_bits = ns * stride
    seed = uniform_bits(seed_bits, c["seed_seed"])
    # The permutation comes from the library's keyed shuffle (no d_assign).
    sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, S.SAMPLE_PERMUTE,
                                 key=c["perm_key"])
    out, tot, st = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, to_dev(seed),
                                  seed_bits, m, out_rule=S.OUT_FIXED, out_a=m,
                                  seed_stride=stride, status=st,
                                  reset_status=False)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_PERMUTE, assign=perm)
    want, wtot = orc.hash_batch(osub, oln, owo, np.full(ns, m, np.uint64),
                                seed, seed_bits, stride, m)
    assert int(tot.item()) == wtot == ns * m
    assert np.array_equal(to_host(out)[: want.size], want)


def _sampled_rows(rng, lens, mlens, k):
    js = rng.integers(0, len(lens), size=k)
    out = []
    for j in js:
        mj = int(mlens[j])
        if mj == 0:
            continue
        r = int(rng.integers(0, mj))
        out.append((int(j), r))
    # tile edges: first/last rows of the first and last sub-blocks
    for j in (0, len(lens) - 1):
        for r in (0, 1, 31, 32, 4095, 4096, int(mlens[j]) - 1):
            if 0 <= r < int(mlens[j]):
                out.append((j, r))
    return out


def test_batched_workload_full_size(ctx, S, orc):
    """2^28 Bernoulli(0.3) bits, i.i.d. over 2048 sub-blocks, floor(0.4 n_j)
    output bits, shared seed: the sampling output is compared in full, the
    hash on 400 sampled rows plus tile-edge rows."""
    import torch
    c = config("batched")
    n, ns = c["n_bits"], c["n_sub"]
    a = bernoulli_bits(n, c["p"], c["input_seed"])
    sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, S.SAMPLE_IID,
                                 key=c["sample_key"])
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID,
                                   key=c["sample_key"])
    assert np.array_equal(to_host(ln)[:ns], oln)
    assert np.array_equal(to_host(wo)[:ns], owo)
    gsub = to_host(sub)[: osub.size]
    assert np.array_equal(gsub, osub), first_diff(gsub, osub)
    om = orc.out_lengths(oln, orc.OUT_RATIO, c["out_a"], c["out_b"])
    cap = int(om.max())
    seed_bits = int(oln.max()) + cap - 1
    seed = uniform_bits(seed_bits, c["seed_seed"])
    out, tot, st = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, to_dev(seed),
                                  seed_bits, cap, out_rule=S.OUT_RATIO,
                                  out_a=c["out_a"], out_b=c["out_b"])
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert int(tot.item()) == int(om.sum())
    got = to_host(out)
    ooff = np.concatenate([[0], np.cumsum(om)[:-1]]).astype(np.int64)
    rng = np.random.default_rng(7)
    for j, r in _sampled_rows(rng, oln, om, 400):
        xj = osub[int(owo[j]):]
        want = orc.toeplitz_rowwin(xj, int(oln[j]), seed, seed_bits, 0, cap, r)
        assert bit(got, int(ooff[j]) + r) == want, (j, r)
    total = int(om.sum())
    tail = got[total // 64:]
    if total % 64:
        assert int(tail[0]) >> (total % 64) == 0


def test_single_block_workload_full_size(ctx, S, orc):
    """n = 2^24 uniform bits hashed to m = 2^23 bits: 160 sampled rows plus
    tile-edge rows against the oracle."""
    c = config("single")
    n, m = c["n_bits"], c["out_a"]
    x = uniform_bits(n, c["input_seed"])
    seed = uniform_bits(n + m - 1, c["seed_seed"])
    got = gpu_hash_one(ctx, S, x, n, seed, n + m - 1, m)
    rng = np.random.default_rng(8)
    rows = sorted(set([int(v) for v in rng.integers(0, m, size=160)] +
                      [0, 1, 31, 32, 4095, 4096, 8191, m - 4096, m - 1]))
    for r in rows:
        assert bit(got, r) == orc.toeplitz_rowwin(x, n, seed, n + m - 1, 0, m,
                                                  r), r
