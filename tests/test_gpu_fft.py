"""GPU parity of the FFT hash (shared seed): the middle product by
double-precision FFTs, rounded and parity-taken, must equal the oracle bit
for bit (tolerance 0), and equal the VALU and matrix-core kernels."""

import numpy as np
import pytest

from tests.gpu_util import first_diff, to_dev, to_dev_u32, to_host
from workloads import bernoulli_bits, config, permutation, uniform_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02856_amd import ssbh
    c = ssbh.Context(0)
    yield c
    c.close()


def fft_hash(ctx, sub, ln, wo, ns, seed, seed_bits, cap, chunk=0, **kw):
    import torch
    from paper_2308_02856_amd import ssbh
    ctx.set_fft_schedule(chunk)
    try:
        out, tot, st = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed,
                                      seed_bits, cap, kernel=ssbh.K_FFT, **kw)
        torch.cuda.synchronize()
    finally:
        ctx.set_fft_schedule(0)
    assert int(st.item()) == 0, ssbh.status_name(int(st.item()))
    return to_host(out), int(tot.item())


@pytest.mark.parametrize("n,ns,m", [(4096, 8, 2048), (1000, 7, 999),
                                    (3000, 1, 777), (65, 3, 64),
                                    (10000, 33, 4096), (200, 5, 900)])
def test_equal_blocks_match_oracle(ctx, orc, n, ns, m):
    from paper_2308_02856_amd import ssbh
    N = n * ns
    a = uniform_bits(N, n + ns + 1)
    perm = permutation(N, m + 1)
    sub, ln, wo, st = ctx.sample(to_dev(a), N, ns, ssbh.SAMPLE_PERMUTE,
                                 assign=to_dev_u32(perm))
    seed_bits = n + m - 1 + 5
    seed = uniform_bits(seed_bits, 17 + m)
    got, tot = fft_hash(ctx, sub, ln, wo, ns, to_dev(seed), seed_bits, m,
                        out_rule=ssbh.OUT_FIXED, out_a=m)
    osub, oln, owo, _ = orc.sample(a, N, ns, orc.SAMPLE_PERMUTE, assign=perm)
    want, wtot = orc.hash_batch(osub, oln, owo, np.full(ns, m, np.uint64),
                                seed, seed_bits, 0, m)
    assert tot == wtot
    assert np.array_equal(got[: want.size], want), first_diff(got[: want.size], want)


@pytest.mark.parametrize("N,ns,chunk", [((1 << 20) + 999, 300, 0),
                                        ((1 << 20) + 999, 300, 7),
                                        (200000, 9, 1), (1 << 17, 1, 0),
                                        (5000, 64, 3)])
def test_uneven_blocks_match_oracle_valu_and_mfma(ctx, orc, N, ns, chunk):
    import torch
    from paper_2308_02856_amd import ssbh
    a = bernoulli_bits(N, 0.3, N % 1009)
    key = 0x3141 + ns
    sub, ln, wo, st = ctx.sample(to_dev(a), N, ns, ssbh.SAMPLE_IID, key=key)
    osub, oln, owo, _ = orc.sample(a, N, ns, orc.SAMPLE_IID, key=key)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 2, 5)
    cap = int(om.max()) + 11
    seed_bits = int(oln.max()) + cap - 1 + 3
    seed = uniform_bits(seed_bits, 77)
    kw = dict(out_rule=ssbh.OUT_RATIO, out_a=2, out_b=5)
    got, tot = fft_hash(ctx, sub, ln, wo, ns, to_dev(seed), seed_bits, cap,
                        chunk=chunk, **kw)
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed, seed_bits, 0, cap)
    assert tot == wtot
    assert np.array_equal(got[: want.size], want), first_diff(got[: want.size], want)
    for kern in (ssbh.K_VALU, ssbh.K_MFMA_I8):
        out, _, st2 = ctx.hash_batch(sub, sub.numel(), ln, wo, ns,
                                     to_dev(seed), seed_bits, cap,
                                     kernel=kern, **kw)
        torch.cuda.synchronize()
        assert int(st2.item()) == 0
        assert np.array_equal(to_host(out), got), kern


@pytest.mark.parametrize("indep", [False, True])
def test_empty_and_degenerate_sub_blocks(ctx, orc, indep):
    """Empty sub-blocks, m_j = 0 and m_j > n_j, from explicit lengths, with
    a shared seed and with independent seeds (complex floats between the
    passes at this length)."""
    import torch
    from paper_2308_02856_amd import ssbh
    lens = np.array([0, 5, 64, 0, 1000, 3, 700], dtype=np.uint64)
    outl = np.array([4, 0, 100, 0, 333, 9, 1], dtype=np.uint64)
    words = (lens + 63) // 64
    wo = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    sub = uniform_bits(int(words.sum()) * 64, 5)
    for j in range(len(lens)):          # clear the bits past n_j
        r = int(lens[j]) % 64
        if r and words[j]:
            sub[int(wo[j] + words[j] - 1)] &= np.uint64((1 << r) - 1)
    cap = int(outl.max())
    ns = len(lens)
    stride = int(lens.max()) + cap - 1 if indep else 0
    seed_bits = ns * stride if indep else int(lens.max()) + cap - 1
    seed = uniform_bits(seed_bits, 6)
    dl = torch.from_numpy(outl.view(np.int64)).cuda()
    got, tot = fft_hash(ctx, to_dev(sub), to_dev(lens), to_dev(wo), ns,
                        to_dev(seed), seed_bits, cap,
                        out_rule=ssbh.OUT_EXPLICIT, out_len=dl,
                        seed_stride=stride)
    if indep:
        assert ctx.last_schedule().endswith(":f32")
    want, wtot = orc.hash_batch(sub, lens, wo, outl, seed, seed_bits, stride, cap)
    assert tot == wtot
    assert np.array_equal(got[: want.size], want)


def test_rejects_long_seeds_and_short_strides(ctx):
    """Seeds (or seed strides) past 2^31 are refused on the host; a stride
    below n_max + m_cap - 1 whose transform cannot hold a sub-block gives
    SSBH_E_UNSUPPORTED on the device."""
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns = 4096, 4
    sub = to_dev(uniform_bits(n, 1))
    ln = torch.full((ns,), n // ns, dtype=torch.int64, device="cuda")
    wo = torch.arange(ns, dtype=torch.int64, device="cuda") * (n // ns // 64)
    seed = to_dev(uniform_bits(1 << 20, 2))
    with pytest.raises(ssbh.SsbhError) as e:
        ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed, (1 << 31) + 1, 100,
                       out_rule=ssbh.OUT_FIXED, out_a=100, kernel=ssbh.K_FFT)
    assert e.value.status == ssbh.E_UNSUPPORTED
    with pytest.raises(ssbh.SsbhError) as e:
        ctx.hash_batch(sub, sub.numel(), ln, wo, 1, seed, 1 << 20, 100,
                       out_rule=ssbh.OUT_FIXED, out_a=100,
                       seed_stride=(1 << 31) + 1, kernel=ssbh.K_FFT)
    assert e.value.status == ssbh.E_UNSUPPORTED
    # n_j = 5000, m = 100: n + m - 1 = 5099 > 4096 = the length for a
    # stride of 2000 (overlapping seeds, legal for the quadratic kernels).
    big = to_dev(uniform_bits(4 * 5000, 3))
    ln2 = torch.full((2,), 5000, dtype=torch.int64, device="cuda")
    wo2 = torch.tensor([0, 79], dtype=torch.int64, device="cuda")
    out, tot, st = ctx.hash_batch(big, big.numel(), ln2, wo2, 2, seed, 1 << 20,
                                  100, out_rule=ssbh.OUT_FIXED, out_a=100,
                                  seed_stride=2000, kernel=ssbh.K_FFT)
    torch.cuda.synchronize()
    assert int(st.item()) == ssbh.E_UNSUPPORTED


@pytest.mark.parametrize("ns,n,m,extra", [(1, 5000, 1200, 0), (5, 30000, 9000, 7),
                                          (4, 100000, 37000, 64), (7, 1000, 999, 3)])
def test_independent_seeds_match_oracle_and_valu(ctx, orc, ns, n, m, extra):
    """Seed stride S = n_max + m - 1 + extra (the paper's independent seeds):
    one transform per sub-block carrying its seed window and its bits; equal
    to the oracle and to the VALU kernel on every bit."""
    import torch
    from paper_2308_02856_amd import ssbh
    N = n * ns + 333
    a = uniform_bits(N, ns * 7 + n)
    key = 0x5EED + ns
    sub, ln, wo, st = ctx.sample(to_dev(a), N, ns, ssbh.SAMPLE_IID, key=key)
    osub, oln, owo, _ = orc.sample(a, N, ns, orc.SAMPLE_IID, key=key)
    S = int(oln.max()) + m - 1 + extra
    seed_bits = ns * S
    seed = uniform_bits(seed_bits, n + m)
    kw = dict(out_rule=ssbh.OUT_FIXED, out_a=m, seed_stride=S)
    got, tot = fft_hash(ctx, sub, ln, wo, ns, to_dev(seed), seed_bits, m, **kw)
    want, wtot = orc.hash_batch(osub, oln, owo, np.full(ns, m, np.uint64),
                                seed, seed_bits, S, m)
    assert tot == wtot
    assert np.array_equal(got[: want.size], want), first_diff(got[: want.size], want)
    out, tot2, st2 = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, to_dev(seed),
                                    seed_bits, m, kernel=ssbh.K_VALU, **kw)
    torch.cuda.synchronize()
    assert int(st2.item()) == 0
    assert np.array_equal(got, to_host(out))


def test_batched_workload_fft_equals_mfma(ctx, orc):
    """Full batched workload (2^28 bits, 2048 sub-blocks): FFT == int8
    matrix cores bit for bit, with the library's chunk and with the two the
    tuner picks between for the benchmark (64 and 85 transforms requested:
    8 launches of 64, and 7 of 74 + ... + 68), plus sampled rows against the
    oracle."""
    import torch
    from paper_2308_02856_amd import ssbh
    c = config("batched")
    n, ns = c["n_bits"], c["n_sub"]
    a = bernoulli_bits(n, c["p"], c["input_seed"])
    sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, ssbh.SAMPLE_IID,
                                 key=c["sample_key"])
    torch.cuda.synchronize()
    lens = to_host(ln)[:ns].astype(np.int64)
    mlen = lens * 2 // 5
    cap = int(mlen.max())
    seed_bits = int(lens.max()) + cap - 1
    seed_h = uniform_bits(seed_bits, c["seed_seed"])
    seed = to_dev(seed_h)
    kw = dict(out_rule=ssbh.OUT_RATIO, out_a=2, out_b=5)
    out, tot2, st2 = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed,
                                    seed_bits, cap, kernel=ssbh.K_MFMA_I8, **kw)
    torch.cuda.synchronize()
    assert int(st2.item()) == 0
    ref = to_host(out)
    for chunk in (0, 64, 85):
        got, tot = fft_hash(ctx, sub, ln, wo, ns, seed, seed_bits, cap,
                            chunk=chunk, **kw)
        assert tot == int(tot2.item())
        assert np.array_equal(got, ref), (chunk, first_diff(got, ref))
    # Sampled rows against the oracle (row windows, one row at a time).
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID,
                                   key=c["sample_key"])
    ooff = np.concatenate([[0], np.cumsum(mlen)[:-1]])
    rng = np.random.default_rng(4)
    for _ in range(40):
        j = int(rng.integers(0, ns))
        r = int(rng.integers(0, int(mlen[j])))
        want = orc.toeplitz_rowwin(osub[int(owo[j]):], int(oln[j]), seed_h,
                                   seed_bits, 0, cap, r)
        k = int(ooff[j]) + r
        assert ((int(got[k >> 6]) >> (k & 63)) & 1) == want, (j, r)


@pytest.mark.parametrize("n,ns", [((1 << 19) + 3, 40), (150001, 1)])
def test_fft_graph_pipeline_replays(ctx, orc, n, ns):
    """Sampling and the FFT hash captured in a graph: every replay gives the
    oracle's output (40 sub-blocks with a shared seed: the packed layout;
    one sub-block: the joint transform with floats between the passes)."""
    import torch
    from paper_2308_02856_amd import ssbh
    a = bernoulli_bits(n, 0.5, 91)
    key = 0x99
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=key)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 1, 3)
    cap = int(om.max())
    seed_bits = int(oln.max()) + cap - 1
    seed = uniform_bits(seed_bits, 92)
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed, seed_bits, 0, cap)
    sub_cap = (n + 63) // 64 + ns
    sub = torch.empty(sub_cap, dtype=torch.int64, device="cuda")
    ln = torch.empty(ns, dtype=torch.int64, device="cuda")
    wo = torch.empty(ns, dtype=torch.int64, device="cuda")
    out = torch.empty((wtot + 63) // 64, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pipe = ctx.pipeline(d_in=to_dev(a), n_bits=n, n_sub=ns,
                        mode=ssbh.SAMPLE_IID, sample_key=key, d_sub=sub,
                        sub_capacity_words=sub_cap, d_len=ln, d_word_off=wo,
                        out_rule=ssbh.OUT_RATIO, out_a=1, out_b=3,
                        d_seed=to_dev(seed), seed_bits=seed_bits, m_cap=cap,
                        kernel=ssbh.K_FFT, d_out=out, out_capacity_bits=wtot,
                        d_out_total_bits=tot, d_status=st)
    for _ in range(3):
        out.fill_(-1)
        torch.cuda.synchronize()
        pipe.launch()
        torch.cuda.synchronize()
        assert int(st.item()) == 0 and int(tot.item()) == wtot
        assert np.array_equal(to_host(out)[: want.size], want)
    pipe.close()


LENGTHS = [4096, 8192, 12288, 16384, 24576, 32768, 49152, 65536, 98304,
           131072, 196608, 262144, 393216, 524288, 786432, 1048576, 1 << 25,
           3 << 24]


@pytest.mark.parametrize("L", LENGTHS)
def test_every_transform_length(ctx, orc, L):
    """Seeds that select transform lengths with two, three and four levels
    (2^k and 3 * 2^k): FFT == VALU kernel on every bit, and sampled rows ==
    the oracle."""
    import torch
    from paper_2308_02856_amd import ssbh
    ns = 6
    seed_bits = L - 3                       # selects exactly this length
    lens = np.array([seed_bits // 2 - 7 * j for j in range(ns)], dtype=np.uint64)
    M = int(seed_bits - int(lens.max()) + 1)            # n_max + M - 1 = seed_bits
    outl = np.array([M - 11 * j for j in range(ns)], dtype=np.uint64)
    words = (lens + 63) // 64
    wo = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    sub = uniform_bits(int(words.sum()) * 64, L)
    for j in range(ns):
        r = int(lens[j]) % 64
        if r:
            sub[int(wo[j] + words[j] - 1)] &= np.uint64((1 << r) - 1)
    seed = uniform_bits(seed_bits, L + 1)
    dl = torch.from_numpy(outl.view(np.int64)).cuda()
    args = (to_dev(sub), sub.size, to_dev(lens), to_dev(wo), ns, to_dev(seed),
            seed_bits, M)
    kw = dict(out_rule=ssbh.OUT_EXPLICIT, out_len=dl)
    got, tot = fft_hash(ctx, args[0], args[2], args[3], ns, args[5],
                        seed_bits, M, **kw)
    assert ctx.last_schedule().endswith(":L%d" % L)
    out, tot2, st = ctx.hash_batch(*args, kernel=ssbh.K_VALU, **kw)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(tot2.item()) == tot
    assert np.array_equal(got, to_host(out))
    ooff = np.concatenate([[0], np.cumsum(outl)[:-1]])
    rng = np.random.default_rng(L)
    for _ in range(12):
        j = int(rng.integers(0, ns))
        r = int(rng.integers(0, int(outl[j])))
        want = orc.toeplitz_rowwin(sub[int(wo[j]):], int(lens[j]), seed,
                                   seed_bits, 0, M, r)
        k = int(ooff[j]) + r
        assert ((int(got[k >> 6]) >> (k & 63)) & 1) == want, (j, r)


@pytest.mark.parametrize("density", [0.05, 0.5, 0.95])
def test_seed_density_stays_exact(ctx, density):
    """Sparse, half-dense and dense seeds (the error bound grows with the
    seed's popcount) all give the VALU kernel's bits."""
    import torch
    from paper_2308_02856_amd import ssbh
    ns = 10
    seed_bits = 190000
    lens = np.array([95000 - 313 * j for j in range(ns)], dtype=np.uint64)
    M = seed_bits - int(lens.max()) + 1
    outl = np.array([M - 97 * j for j in range(ns)], dtype=np.uint64)
    words = (lens + 63) // 64
    wo = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    sub = bernoulli_bits(int(words.sum()) * 64, 0.5, 3)
    for j in range(ns):
        r = int(lens[j]) % 64
        if r:
            sub[int(wo[j] + words[j] - 1)] &= np.uint64((1 << r) - 1)
    seed = bernoulli_bits(seed_bits, density, 4)
    dl = torch.from_numpy(outl.view(np.int64)).cuda()
    kw = dict(out_rule=ssbh.OUT_EXPLICIT, out_len=dl)
    d_sub, d_len, d_wo, d_seed = to_dev(sub), to_dev(lens), to_dev(wo), to_dev(seed)
    got, tot = fft_hash(ctx, d_sub, d_len, d_wo, ns, d_seed, seed_bits, M, **kw)
    out, tot2, st = ctx.hash_batch(d_sub, d_sub.numel(), d_len, d_wo, ns, d_seed,
                                   seed_bits, M, kernel=ssbh.K_VALU, **kw)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(tot2.item()) == tot
    assert np.array_equal(got, to_host(out))


def test_single_block_workload_three_levels(ctx, orc):
    """The single-block workload (n = 2^24 -> m = 2^23, seed n + m - 1 bits)
    runs as a three-level transform of 3 * 2^23 points: equal to the VALU
    kernel on every bit and to the oracle on sampled rows."""
    import torch
    from paper_2308_02856_amd import ssbh
    c = config("single")
    n, m = c["n_bits"], c["out_a"]
    x = uniform_bits(n, c["input_seed"])
    seed_bits = n + m - 1
    seed_h = uniform_bits(seed_bits, c["seed_seed"])
    d_x, seed = to_dev(x), to_dev(seed_h)
    ln = torch.tensor([n], dtype=torch.int64, device="cuda")
    wo = torch.zeros(1, dtype=torch.int64, device="cuda")
    kw = dict(out_rule=ssbh.OUT_FIXED, out_a=m)
    got, tot = fft_hash(ctx, d_x, ln, wo, 1, seed, seed_bits, m, **kw)
    assert ctx.last_schedule().endswith(":L%d" % (3 << 23))
    out, tot2, st = ctx.hash_batch(d_x, d_x.numel(), ln, wo, 1, seed,
                                   seed_bits, m, kernel=ssbh.K_VALU, **kw)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and tot == int(tot2.item()) == m
    assert np.array_equal(got, to_host(out))
    rng = np.random.default_rng(24)
    for r in [0, 1, m - 1] + [int(v) for v in rng.integers(0, m, 10)]:
        want = orc.toeplitz_rowwin(x, n, seed_h, seed_bits, 0, m, r)
        assert ((int(got[r >> 6]) >> (r & 63)) & 1) == want, r


@pytest.mark.parametrize("n,m,want_fft,indep", [(1 << 16, 1 << 15, True, False),
                                                (4000, 2000, False, False),
                                                (1 << 16, 1 << 15, True, True),
                                                (4000, 2000, False, True)])
def test_untuned_auto_picks_fft_for_long_blocks(n, m, want_fft, indep):
    """Without a tuned entry, AUTO takes the FFT when the quadratic work is
    well above the transform's (n m >= 1024 L log2 L / sub-blocks per
    transform), for a shared seed and for independent seeds alike, and gives
    the VALU kernel's bits either way."""
    import torch
    from paper_2308_02856_amd import ssbh
    ctx = ssbh.Context(0)
    try:
        ns = 4
        words = (n + 63) // 64
        sub = uniform_bits(ns * words * 64, n)
        lens = np.full(ns, n, np.uint64)
        wo = (np.arange(ns) * words).astype(np.uint64)
        stride = n + m - 1 if indep else 0
        seed_bits = (ns if indep else 1) * (n + m - 1)
        seed = to_dev(uniform_bits(seed_bits, m))
        args = (to_dev(sub), sub.size, to_dev(lens), to_dev(wo), ns, seed,
                seed_bits, m)
        kw = dict(out_rule=ssbh.OUT_FIXED, out_a=m, seed_stride=stride)
        out, tot, st = ctx.hash_batch(*args, kernel=ssbh.K_AUTO, **kw)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        assert ctx.last_schedule().startswith("fft") == want_fft
        ref, tot2, st2 = ctx.hash_batch(*args, kernel=ssbh.K_VALU, **kw)
        torch.cuda.synchronize()
        assert int(st2.item()) == 0 and int(tot.item()) == int(tot2.item())
        assert np.array_equal(to_host(out), to_host(ref))
    finally:
        ctx.close()


def test_four_level_single_block_960_mbit(ctx, orc):
    """Table I's fourth input size as one block: n = 960.40 Mbit hashed to
    m = 74.406 Mbit (seed n + m - 1 bits, transform length 2^30, four
    levels); sampled rows, including both ends, against the oracle."""
    import torch
    from paper_2308_02856_amd import ssbh
    n, m = 960_400_000, 74_406_000
    x = uniform_bits(n, 2960)
    seed_bits = n + m - 1
    seed_h = uniform_bits(seed_bits, 2961)
    d_x, seed = to_dev(x), to_dev(seed_h)
    ln = torch.tensor([n], dtype=torch.int64, device="cuda")
    wo = torch.zeros(1, dtype=torch.int64, device="cuda")
    got, tot = fft_hash(ctx, d_x, ln, wo, 1, seed, seed_bits, m,
                        out_rule=ssbh.OUT_FIXED, out_a=m)
    assert ctx.last_schedule().endswith(":L%d" % (1 << 30)) and tot == m
    del d_x, seed
    torch.cuda.empty_cache()
    rng = np.random.default_rng(960)
    for r in [0, 1, 63, 64, m - 1] + [int(v) for v in rng.integers(0, m, 6)]:
        want = orc.toeplitz_rowwin(x, n, seed_h, seed_bits, 0, m, r)
        assert ((int(got[r >> 6]) >> (r & 63)) & 1) == want, r


@pytest.mark.parametrize("L", LENGTHS)
def test_every_transform_length_independent(ctx, orc, L):
    """Independent seeds (stride S = L - 3 selects the length; sub-block j's
    seed window starts at bit jS) with two, three and four levels: FFT ==
    VALU kernel on every bit, and sampled rows == the oracle."""
    import torch
    from paper_2308_02856_amd import ssbh
    ns = 5
    S = L - 3
    lens = np.array([S // 2 - 7 * j for j in range(ns)], dtype=np.uint64)
    M = int(S - int(lens.max()) + 1)                   # n_max + M - 1 = S
    outl = np.array([M - 11 * j for j in range(ns)], dtype=np.uint64)
    words = (lens + 63) // 64
    wo = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    sub = uniform_bits(int(words.sum()) * 64, L + 5)
    for j in range(ns):
        r = int(lens[j]) % 64
        if r:
            sub[int(wo[j] + words[j] - 1)] &= np.uint64((1 << r) - 1)
    seed_bits = ns * S
    seed = uniform_bits(seed_bits, L + 6)
    dl = torch.from_numpy(outl.view(np.int64)).cuda()
    args = (to_dev(sub), sub.size, to_dev(lens), to_dev(wo), ns, to_dev(seed),
            seed_bits, M)
    kw = dict(out_rule=ssbh.OUT_EXPLICIT, out_len=dl, seed_stride=S)
    got, tot = fft_hash(ctx, args[0], args[2], args[3], ns, args[5],
                        seed_bits, M, **kw)
    sched = ctx.last_schedule()
    assert (":L%d" % L) in sched
    assert sched.endswith(":f32") == (L <= 1 << 18)
    out, tot2, st = ctx.hash_batch(*args, kernel=ssbh.K_VALU, **kw)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(tot2.item()) == tot
    assert np.array_equal(got, to_host(out)), first_diff(got, to_host(out))
    ooff = np.concatenate([[0], np.cumsum(outl)[:-1]])
    rng = np.random.default_rng(L + 1)
    for _ in range(12):
        j = int(rng.integers(0, ns))
        r = int(rng.integers(0, int(outl[j])))
        want = orc.toeplitz_rowwin(sub[int(wo[j]):], int(lens[j]), seed,
                                   seed_bits, j * S, M, r)
        k = int(ooff[j]) + r
        assert ((int(got[k >> 6]) >> (k & 63)) & 1) == want, (j, r)


def test_two_streams_of_chunks_on_a_caller_stream(ctx, orc):
    """Chunks of one transform each alternate between the caller's stream and
    the library's second stream: two calls back to back on a non-default
    torch stream, then the caller's own copy of the output on that stream
    (no host wait between), equal the oracle and the one-chunk result."""
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns = 300001, 24
    a = bernoulli_bits(n, 0.4, 93)
    key = 0x515
    sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, ssbh.SAMPLE_IID, key=key)
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=key)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 2, 5)
    cap = int(om.max())
    seed_bits = int(oln.max()) + cap - 1
    seed = uniform_bits(seed_bits, 94)
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed, seed_bits, 0, cap)
    d_seed = to_dev(seed)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    kw = dict(out_rule=ssbh.OUT_RATIO, out_a=2, out_b=5, kernel=ssbh.K_FFT)
    ctx.set_fft_schedule(1)
    try:
        with torch.cuda.stream(side):
            o1, t1, s1 = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, d_seed,
                                        seed_bits, cap, **kw)
            o2, t2, s2 = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, d_seed,
                                        seed_bits, cap, **kw)
            c1, c2 = o1.clone(), o2.clone()
        side.synchronize()
    finally:
        ctx.set_fft_schedule(0)
    assert int(s1.item()) == 0 and int(s2.item()) == 0
    assert int(t1.item()) == wtot and int(t2.item()) == wtot
    for c in (c1, c2):
        assert np.array_equal(to_host(c)[: want.size], want)
    one, _ = fft_hash(ctx, sub, ln, wo, ns, d_seed, seed_bits, cap, chunk=64,
                      out_rule=ssbh.OUT_RATIO, out_a=2, out_b=5)
    assert np.array_equal(one[: want.size], want)


def test_fft_graph_pipeline_many_chunks(ctx, orc):
    """A captured pipeline with one transform per chunk (the capture keeps
    every chunk on the pipeline's stream): replays equal the oracle."""
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns = (1 << 18) + 5, 12
    a = bernoulli_bits(n, 0.5, 95)
    key = 0x9A
    osub, oln, owo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=key)
    om = orc.out_lengths(oln, orc.OUT_RATIO, 1, 3)
    cap = int(om.max())
    seed_bits = int(oln.max()) + cap - 1
    seed = uniform_bits(seed_bits, 96)
    want, wtot = orc.hash_batch(osub, oln, owo, om, seed, seed_bits, 0, cap)
    sub_cap = (n + 63) // 64 + ns
    sub = torch.empty(sub_cap, dtype=torch.int64, device="cuda")
    ln = torch.empty(ns, dtype=torch.int64, device="cuda")
    wo = torch.empty(ns, dtype=torch.int64, device="cuda")
    out = torch.empty((wtot + 63) // 64, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.set_fft_schedule(1)
    try:
        pipe = ctx.pipeline(d_in=to_dev(a), n_bits=n, n_sub=ns,
                            mode=ssbh.SAMPLE_IID, sample_key=key, d_sub=sub,
                            sub_capacity_words=sub_cap, d_len=ln,
                            d_word_off=wo, out_rule=ssbh.OUT_RATIO, out_a=1,
                            out_b=3, d_seed=to_dev(seed), seed_bits=seed_bits,
                            m_cap=cap, kernel=ssbh.K_FFT, d_out=out,
                            out_capacity_bits=wtot, d_out_total_bits=tot,
                            d_status=st)
    finally:
        ctx.set_fft_schedule(0)
    for _ in range(3):
        out.fill_(-1)
        torch.cuda.synchronize()
        pipe.launch()
        torch.cuda.synchronize()
        assert int(st.item()) == 0 and int(tot.item()) == wtot
        assert np.array_equal(to_host(out)[: want.size], want)
    pipe.close()


def _all_ones_subs(lens):
    words = (lens + 63) // 64
    wo = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    sub = np.full(int(words.sum()), np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    for j in range(lens.size):
        r = int(lens[j]) % 64
        if r:
            sub[int(wo[j] + words[j] - 1)] = np.uint64((1 << r) - 1)
    return sub, wo


def test_float_storage_worst_case_all_ones(ctx):
    """Independent seeds at the longest transform that keeps complex floats
    between the passes (L = 2^18), with every seed and input bit set: |z|^2
    = L + n_j (the real part holds L seed bits), near the 2 L the rounding
    bound covers.  Every
    entry of T_j x_j is then n_j, so every output bit of sub-block j is
    n_j mod 2; the float and double storage give exactly that."""
    import torch
    from paper_2308_02856_amd import ssbh
    S = 1 << 18
    M = 4096
    lens = np.array([S - M + 1 - j for j in range(3)], dtype=np.uint64)
    ns = lens.size
    sub, wo = _all_ones_subs(lens)
    seed_bits = ns * S
    seed = np.full(seed_bits // 64, np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    want = np.concatenate([np.full(M, int(n) & 1, dtype=np.uint8) for n in lens])
    args = (to_dev(sub), sub.size, to_dev(lens), to_dev(wo), ns, to_dev(seed),
            seed_bits, M)
    kw = dict(out_rule=ssbh.OUT_FIXED, out_a=M, seed_stride=S, kernel=ssbh.K_FFT)
    for bits, suffix in ((0, ":f32"), (32, ":f32"), (64, ":L%d" % S)):
        ctx.set_fft_storage(bits)
        try:
            out, tot, st = ctx.hash_batch(*args, **kw)
            torch.cuda.synchronize()
            sched = ctx.last_schedule()
        finally:
            ctx.set_fft_storage(0)
        assert int(st.item()) == 0, ssbh.status_name(int(st.item()))
        assert sched.endswith(suffix), (bits, sched)
        assert int(tot.item()) == ns * M
        got = np.unpackbits(to_host(out).view(np.uint8), bitorder="little")[: ns * M]
        assert np.array_equal(got, want), (bits, first_diff(got, want))


@pytest.mark.parametrize("ns,lmax,m", [(6, 120000, 48000), (33, 5000, 1700)])
def test_float_and_double_storage_agree_with_oracle(ctx, orc, ns, lmax, m):
    """Independent seeds, uneven sub-blocks: the hash with complex floats and
    with complex doubles between the passes both equal the oracle bit for
    bit (float storage is the library's choice at these lengths)."""
    import torch
    from paper_2308_02856_amd import ssbh
    rng = np.random.default_rng(ns + lmax)
    lens = rng.integers(lmax // 2, lmax + 1, ns).astype(np.uint64)
    lens[0] = lmax
    words = (lens + 63) // 64
    wo = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    sub = bernoulli_bits(int(words.sum()) * 64, 0.3, ns)
    for j in range(ns):
        r = int(lens[j]) % 64
        if r:
            sub[int(wo[j] + words[j] - 1)] &= np.uint64((1 << r) - 1)
    S = lmax + m - 1
    seed_bits = ns * S
    seed = uniform_bits(seed_bits, lmax + 1)
    want, wtot = orc.hash_batch(sub, lens, wo, np.full(ns, m, np.uint64),
                                seed, seed_bits, S, m)
    args = (to_dev(sub), sub.size, to_dev(lens), to_dev(wo), ns, to_dev(seed),
            seed_bits, m)
    kw = dict(out_rule=ssbh.OUT_FIXED, out_a=m, seed_stride=S, kernel=ssbh.K_FFT)
    for bits in (0, 64, 32):
        ctx.set_fft_storage(bits)
        try:
            out, tot, st = ctx.hash_batch(*args, **kw)
            torch.cuda.synchronize()
            sched = ctx.last_schedule()
        finally:
            ctx.set_fft_storage(0)
        assert int(st.item()) == 0, ssbh.status_name(int(st.item()))
        assert sched.endswith(":f32") == (bits != 64), sched
        got = to_host(out)
        assert int(tot.item()) == wtot
        assert np.array_equal(got[: want.size], want), (bits, first_diff(got[: want.size], want))


def test_float_storage_refused_where_unbounded(ctx):
    """Float storage is refused with a shared seed and above L = 2^18 (host
    error SSBH_E_UNSUPPORTED), and the setter takes only 0, 32 and 64."""
    import torch
    from paper_2308_02856_amd import ssbh
    with pytest.raises(ssbh.SsbhError) as e:
        ctx.set_fft_storage(16)
    assert e.value.status == ssbh.E_INVAL
    n, ns = 4096, 4
    sub = to_dev(uniform_bits(n, 1))
    ln = torch.full((ns,), n // ns, dtype=torch.int64, device="cuda")
    wo = torch.arange(ns, dtype=torch.int64, device="cuda") * (n // ns // 64)
    seed = to_dev(uniform_bits(ns * ((1 << 18) + 1), 2))
    ctx.set_fft_storage(32)
    try:
        for stride, seed_bits in ((0, 2000), ((1 << 18) + 1, ns * ((1 << 18) + 1))):
            with pytest.raises(ssbh.SsbhError) as e:
                ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed, seed_bits, 100,
                               out_rule=ssbh.OUT_FIXED, out_a=100,
                               seed_stride=stride, kernel=ssbh.K_FFT)
            assert e.value.status == ssbh.E_UNSUPPORTED, stride
    finally:
        ctx.set_fft_storage(0)


@pytest.mark.parametrize("n,m,ones", [(100000, 40000, False), (1 << 18, 1 << 17, False),
                                      ((1 << 18) - 4095, 4096, True)])
def test_single_sub_block_joint_transform(ctx, orc, n, m, ones):
    """One sub-block with a shared seed takes the joint transform (seed real,
    bits imaginary, one transform, no seed spectrum; complex floats between
    the passes up to L = 2^18): equal to the packed two-per-transform layout
    (forced) and to the oracle bit for bit; with every bit set (ones) each
    output bit is n mod 2."""
    import torch
    from paper_2308_02856_amd import ssbh
    seed_bits = n + m - 1
    if ones:
        x = np.full((n + 63) // 64, np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
        seed = np.full((seed_bits + 63) // 64, np.uint64(0xFFFFFFFFFFFFFFFF),
                       dtype=np.uint64)
        if seed_bits % 64:
            seed[-1] = np.uint64((1 << (seed_bits % 64)) - 1)
    else:
        x = bernoulli_bits(((n + 63) // 64) * 64, 0.5, n)
        seed = uniform_bits(seed_bits, m)
    if n % 64:
        x[-1] &= np.uint64((1 << (n % 64)) - 1)
    lens = np.array([n], dtype=np.uint64)
    wo = np.array([0], dtype=np.uint64)
    args = (to_dev(x), x.size, to_dev(lens), to_dev(wo), 1, to_dev(seed),
            seed_bits, m)
    kw = dict(out_rule=ssbh.OUT_FIXED, out_a=m, kernel=ssbh.K_FFT)
    outs = {}
    for pack in (0, 1):
        ctx.set_fft_packing(pack)
        try:
            out, tot, st = ctx.hash_batch(*args, **kw)
            torch.cuda.synchronize()
            sched = ctx.last_schedule()
        finally:
            ctx.set_fft_packing(0)
        assert int(st.item()) == 0, ssbh.status_name(int(st.item()))
        assert int(tot.item()) == m
        assert (":x1:" if pack == 0 else ":x2:") in sched, sched
        if pack == 0:
            assert sched.endswith(":f32") == (int(sched.split(":L")[1].split(":")[0]) <= 1 << 18)
        outs[pack] = to_host(out)
    assert np.array_equal(outs[0], outs[1]), first_diff(outs[0], outs[1])
    if ones:
        bits = np.unpackbits(outs[0].view(np.uint8), bitorder="little")[:m]
        assert np.all(bits == (n & 1))
    else:
        want, wtot = orc.hash_batch(x, lens, wo, np.array([m], np.uint64),
                                    seed, seed_bits, 0, m)
        assert wtot == m
        assert np.array_equal(outs[0][: want.size], want), first_diff(outs[0][: want.size], want)
