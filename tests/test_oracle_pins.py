"""Pins for the CPU oracle: facts fixed by the paper and by mathematics.

Nothing here re-types the oracle's own formulas.  The Toeplitz product is
pinned by two independent algorithms (carry-less polynomial multiplication on
Python integers, and a float64 FFT correlation with a proven rounding margin),
by closed forms (impulse seed, all-ones input, one output row), by GF(2)
linearity and by diagonal constancy.  Sampling is pinned by published
SplitMix64 outputs, by numpy boolean selection / fancy indexing (library
routines), by the bijection property and by the abort rule of Sec. III.B.
"""

import math
import os

import numpy as np
import pytest

from workloads import (assignment, bernoulli_bits, pack_bits, permutation,
                       uniform_bits, unpack_bits)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------ independent algorithms ---

def seed_window_bits(seed_words, start, length):
    """Bits start .. start+length-1 of a packed seed as a 0/1 array."""
    allbits = unpack_bits(seed_words, seed_words.size * 64)
    return allbits[start:start + length]


def clmul(a: int, b: int) -> int:
    """Carry-less (GF(2)[z]) product of two bit-polynomials held in ints."""
    r = 0
    while b:
        if b & 1:
            r ^= a
        a <<= 1
        b >>= 1
    return r


def toeplitz_by_clmul(xbits, sbits, m, cap):
    """K[r] as the coefficient of z^{n-1+(cap-1-r)} of S(z) * X~(z), where
    S = sum s_k z^k over the seed window and X~ = sum x_c z^{n-1-c}."""
    n = len(xbits)
    S = 0
    for k, b in enumerate(sbits):
        if b:
            S |= 1 << k
    X = 0
    for c, b in enumerate(xbits):
        if b:
            X |= 1 << (n - 1 - c)
    P = clmul(S, X)
    return np.array([(P >> (n - 1 + cap - 1 - r)) & 1 for r in range(m)],
                    dtype=np.uint8)


def toeplitz_by_fft(xbits, sbits, m, cap):
    """Integer correlation by float64 FFT, rounded, reduced mod 2.  The
    rounding residual is asserted below 0.25 so the result is exact."""
    n = len(xbits)
    if n == 0 or m == 0:
        return np.zeros(m, dtype=np.uint8)
    s = np.asarray(sbits, dtype=np.float64)
    x = np.asarray(xbits, dtype=np.float64)[::-1]
    L = 1
    while L < s.size + x.size:
        L *= 2
    conv = np.fft.irfft(np.fft.rfft(s, L) * np.fft.rfft(x, L), L)
    u = cap - 1 - np.arange(m)
    vals = conv[u + n - 1]
    resid = np.abs(vals - np.round(vals)).max()
    assert resid < 0.25, resid
    return (np.round(vals).astype(np.int64) & 1).astype(np.uint8)


def rand_bits(n, seed):
    return unpack_bits(uniform_bits(n, seed), n)


# ------------------------------------------------------------- SplitMix64 ---

def test_splitmix64_published_values(orc):
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) >= 6
    for seed, idx, val in rows:
        assert orc.splitmix64(int(seed), int(idx)) == int(val)


def test_splitmix64_counter_form_equals_sequential(orc):
    for key in (0, 1, 1234567, 2**64 - 1, 0x2308028560000103):
        seq = orc.splitmix64_seq(key, 257)
        cnt = np.array([orc.splitmix64(key, t) for t in range(257)],
                       dtype=np.uint64)
        assert np.array_equal(seq, cnt)


def test_draw_v_power_of_two_takes_top_bits(orc):
    key = 0xABCDEF
    for log2 in (0, 1, 3, 11, 13):
        ns = 1 << log2
        for i in range(200):
            r = orc.splitmix64(key, i // 2)
            u = (r >> 32) if (i & 1) else (r & 0xFFFFFFFF)
            want = (u >> (32 - log2)) if log2 else 0
            assert orc.draw_v(key, i, ns) == want


def test_draw_v_range_and_uniformity(orc):
    ns, n = 7, 70000
    v = orc.assign_iid(n, ns, 99)
    assert v.max() < ns
    counts = np.bincount(v, minlength=ns)
    chi2 = (((counts - n / ns) ** 2) / (n / ns)).sum()
    assert chi2 < 30.0  # 6 dof; p ~ 4e-5


@pytest.mark.parametrize("ns", [3, 7, 13, 1000, 2049, 12345])
def test_draw_v_is_a_monotone_even_range_map(orc, ns):
    """For any N_S (not only powers of two) V_i is a non-decreasing function
    of u_i that spreads [0, 2^32) evenly over [0, N_S) (tests/pin_checks.py;
    a reduction u mod N_S, also uniform, fails it)."""
    from tests.pin_checks import check_v_map
    check_v_map(orc.draw_v, orc.splitmix64, ns,
                count=max(20000, 25 * ns) if ns < 5000 else 20000)


def test_assign_iid_matches_single_draws(orc):
    v = orc.assign_iid(1001, 13, 5)
    assert all(int(v[i]) == orc.draw_v(5, i, 13) for i in range(1001))


def test_seed_from_key(orc):
    s = orc.seed_from_key(77, 200)
    assert s.size == 4
    for t in range(3):
        assert int(s[t]) == orc.splitmix64(77, t)
    assert int(s[3]) == orc.splitmix64(77, 3) & ((1 << 8) - 1)


# ---------------------------------------------------------------- sampling ---

@pytest.mark.parametrize("n,ns", [(1, 1), (10007, 13), (4096, 64), (777, 1),
                                  (5000, 2048)])
def test_partition_equals_boolean_selection(orc, n, ns):
    a = bernoulli_bits(n, 0.3, n + ns)
    v = assignment(n, ns, 1000 + n)
    sub, ln, wo = orc.partition(a, n, v, ns)
    abits = unpack_bits(a, n)
    assert np.array_equal(ln, np.bincount(v, minlength=ns).astype(np.uint64))
    words = (ln + 63) // 64
    assert np.array_equal(wo, np.concatenate([[0], np.cumsum(words)[:-1]])
                          .astype(np.uint64))
    recon = np.zeros(n, dtype=np.uint8)
    for j in range(ns):
        got = unpack_bits(sub[int(wo[j]):int(wo[j] + words[j])],
                          int(words[j]) * 64)
        want = abits[v == j]           # ascending-i selection
        assert np.array_equal(got[:int(ln[j])], want)
        assert not got[int(ln[j]):].any()   # pad bits are zero
        recon[np.nonzero(v == j)[0]] = got[:int(ln[j])]
    assert np.array_equal(recon, abits)     # every bit lands exactly once


def test_sample_iid_is_partition_by_splitmix_assignment(orc):
    n, ns, key = 20000, 37, 0x1234
    a = uniform_bits(n, 3)
    sub, ln, wo, abort = orc.sample(a, n, ns, orc.SAMPLE_IID, key=key)
    sub2, ln2, wo2 = orc.partition(a, n, orc.assign_iid(n, ns, key), ns)
    assert not abort
    assert np.array_equal(sub, sub2) and np.array_equal(ln, ln2)
    assert int(ln.sum()) == n


def test_abort_threshold(orc):
    n, ns = 30000, 16
    a = uniform_bits(n, 4)
    _, ln, _, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=9)
    mx = int(ln.max())
    assert orc.sample(a, n, ns, orc.SAMPLE_IID, key=9, l_ub=mx - 1)[3]
    assert not orc.sample(a, n, ns, orc.SAMPLE_IID, key=9, l_ub=mx)[3]
    assert not orc.sample(a, n, ns, orc.SAMPLE_IID, key=9, l_ub=0)[3]


@pytest.mark.parametrize("n,ns", [(1 << 12, 8), (960, 3), (64 * 5, 5)])
def test_permute_split_equals_fancy_indexing(orc, n, ns):
    a = uniform_bits(n, 11)
    perm = permutation(n, 12)
    assert np.array_equal(np.sort(perm), np.arange(n, dtype=np.uint32))
    sub, ln, wo = orc.permute_split(a, n, perm, ns)
    b = unpack_bits(a, n)[perm]
    L = n // ns
    wl = (L + 63) // 64
    for j in range(ns):
        got = unpack_bits(sub[j * wl:(j + 1) * wl], wl * 64)
        assert np.array_equal(got[:L], b[j * L:(j + 1) * L])
        assert not got[L:].any()
    assert np.all(ln == L)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 64, 1000, 65537])
def test_keyed_permutation_is_a_permutation(orc, n):
    for key in (0, 7, 2**64 - 1):
        perm = orc.permutation(n, key)
        assert perm.dtype == np.uint32 and perm.size == n
        assert np.array_equal(np.sort(perm), np.arange(n, dtype=np.uint32))


def test_keyed_permutation_choices(orc):
    """The exchange index j_i of step i is uniform in [0, i]: it is a
    non-decreasing function of the stream output r_{n-1-i} (pinned by the
    published SplitMix64 values) with j_i / (i+1) within 1/(i+1) of
    r / 2^64.  The last entry is set once, by the first step, so
    perm[n-1] = j_{n-1}."""
    n = 1000
    for i in (1, 2, 5, 999):
        rs, js = [], []
        for key in range(3000):
            r = orc.splitmix64(key, n - 1 - i)
            j = orc.shuffle_choice(key, n, i)
            assert 0 <= j <= i
            assert abs(j / (i + 1) - r / 2.0 ** 64) <= 1.0 / (i + 1)
            rs.append(r)
            js.append(j)
        order = np.argsort(np.array(rs, dtype=np.uint64), kind="stable")
        assert np.all(np.diff(np.array(js)[order]) >= 0)
    for key in range(200):
        for m in (2, 3, 17, 1000):
            assert int(orc.permutation(m, key)[m - 1]) == \
                orc.shuffle_choice(key, m, m - 1)
    # n = 2: the one step swaps exactly when j_1 = 0, i.e. r_0 < 2^63.
    for key in range(200):
        swapped = orc.permutation(2, key).tolist() == [1, 0]
        assert swapped == (orc.splitmix64(key, 0) < 2 ** 63)


@pytest.mark.parametrize("n,keys", [(3, 3000), (4, 6000), (5, 24000)])
def test_keyed_permutation_is_uniform_over_all_orderings(orc, n, keys):
    """Over many keys every one of the n! orderings appears, equally often
    (chi-square; Sattolo's variant, which only makes cycles, or a biased
    exchange index would fail)."""
    counts = {}
    for key in range(keys):
        t = tuple(orc.permutation(n, 0x1000 + 7919 * key).tolist())
        counts[t] = counts.get(t, 0) + 1
    cells = math.factorial(n)
    assert len(counts) == cells
    e = keys / cells
    chi2 = sum((c - e) ** 2 / e for c in counts.values())
    dof = cells - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof) + 10, chi2


def test_permute_split_rejects_indivisible(orc):
    with pytest.raises(ValueError):
        orc.permute_split(uniform_bits(100, 1), 100, permutation(100, 2), 3)


def test_out_lengths(orc):
    ln = np.array([0, 1, 5, 131072, 131073, 2**40 + 3], dtype=np.uint64)
    assert list(orc.out_lengths(ln, orc.OUT_FIXED, 99)) == [99] * 6
    got = orc.out_lengths(ln, orc.OUT_RATIO, 2, 5)
    assert [int(g) for g in got] == [(int(v) * 2) // 5 for v in ln]
    assert int(got[3]) == 52428
    big = orc.out_lengths(np.array([2**62], dtype=np.uint64), orc.OUT_RATIO,
                          3, 7)
    assert int(big[0]) == (2**62 * 3) // 7


# ---------------------------------------------------------------- Toeplitz ---

def oracle_bits(orc, xbits, sbits, m, cap=None, base=0, level=1):
    n = len(xbits)
    cap = m if cap is None else cap
    x = pack_bits(xbits) if n else np.zeros(1, dtype=np.uint64)
    s = pack_bits(sbits) if len(sbits) else np.zeros(1, dtype=np.uint64)
    out = orc.toeplitz(x, n, s, len(sbits), m, base=base, cap=cap,
                       level=level)
    return unpack_bits(out, m)


def test_toeplitz_exhaustive_tiny_against_clmul(orc):
    for n in range(1, 5):
        for m in range(1, 5):
            ls = n + m - 1
            for sv in range(1 << ls):
                sbits = [(sv >> k) & 1 for k in range(ls)]
                for xv in range(1 << n):
                    xbits = [(xv >> k) & 1 for k in range(n)]
                    want = toeplitz_by_clmul(xbits, sbits, m, m)
                    for level in (0, 1):
                        got = oracle_bits(orc, np.array(xbits), np.array(sbits),
                                          m, level=level)
                        assert np.array_equal(got, want), (n, m, sv, xv, level)


@pytest.mark.parametrize("n,m", [(1, 1), (63, 65), (64, 64), (100, 37),
                                 (1000, 1500), (4097, 2049), (3000, 1),
                                 (1, 700)])
def test_toeplitz_against_fft_and_clmul(orc, n, m):
    xbits = rand_bits(n, n * 7 + m)
    sbits = rand_bits(n + m - 1, n * 11 + m)
    want = toeplitz_by_fft(xbits, sbits, m, m)
    assert np.array_equal(want, toeplitz_by_clmul(xbits, sbits, m, m))
    for level in (0, 1):
        assert np.array_equal(oracle_bits(orc, xbits, sbits, m, level=level),
                              want)


def test_toeplitz_large_against_fft(orc):
    n, m = 32768 + 45, 16384 + 13
    xbits = rand_bits(n, 21)
    sbits = rand_bits(n + m - 1, 22)
    got = oracle_bits(orc, xbits, sbits, m, level=1)
    assert np.array_equal(got, toeplitz_by_fft(xbits, sbits, m, m))


def test_toeplitz_seed_offset_and_row_cap(orc):
    # T[r][c] = s[base + c - r + cap - 1]: the block reads the seed window that
    # starts at `base`, and a cap above m selects the top rows of the taller
    # cap x n matrix.
    n, m, cap, base = 777, 300, 450, 1234
    xbits = rand_bits(n, 31)
    sbits = rand_bits(base + n + cap - 1 + 50, 32)
    got = oracle_bits(orc, xbits, sbits, m, cap=cap, base=base, level=1)
    window = sbits[base:base + n + cap - 1]
    want = toeplitz_by_fft(xbits, window, m, cap)
    assert np.array_equal(got, want)
    tall = toeplitz_by_fft(xbits, window, cap, cap)
    assert np.array_equal(got, tall[:m])
    assert np.array_equal(oracle_bits(orc, xbits, sbits, m, cap=cap,
                                      base=base, level=0), want)


def test_toeplitz_closed_forms(orc):
    n, m = 257, 130
    x = rand_bits(n, 41)
    s = rand_bits(n + m - 1, 42)
    z = np.zeros
    assert not oracle_bits(orc, x, z(n + m - 1, np.uint8), m).any()
    assert not oracle_bits(orc, z(n, np.uint8), s, m).any()
    # one output row: inner product of x with the first n seed bits
    got = oracle_bits(orc, x, s[:n], 1)
    assert got[0] == (int(np.dot(x.astype(int), s[:n].astype(int))) & 1)
    # impulse seed e_k shifts the input: K[r] = x[r + k - m + 1]
    for k in (0, m - 1, m + 5, n + m - 2):
        e = z(n + m - 1, np.uint8)
        e[k] = 1
        got = oracle_bits(orc, x, e, m)
        want = np.array([x[r + k - m + 1] if 0 <= r + k - m + 1 < n else 0
                         for r in range(m)], dtype=np.uint8)
        assert np.array_equal(got, want), k
    # identity when m = n and the impulse sits at m - 1
    e = z(2 * n - 1, np.uint8)
    e[n - 1] = 1
    assert np.array_equal(oracle_bits(orc, x, e, n), x)
    # all-ones input: K[r] = P[n+m-1-r] xor P[m-1-r], P = prefix xor of s
    P = np.concatenate([[0], np.bitwise_xor.accumulate(s)]).astype(np.uint8)
    got = oracle_bits(orc, np.ones(n, np.uint8), s, m)
    want = np.array([P[n + m - 1 - r] ^ P[m - 1 - r] for r in range(m)],
                    dtype=np.uint8)
    assert np.array_equal(got, want)


def test_toeplitz_linearity(orc):
    n, m = 999, 321
    a, b = rand_bits(n, 51), rand_bits(n, 52)
    s, t = rand_bits(n + m - 1, 53), rand_bits(n + m - 1, 54)
    assert np.array_equal(oracle_bits(orc, a ^ b, s, m),
                          oracle_bits(orc, a, s, m) ^ oracle_bits(orc, b, s, m))
    assert np.array_equal(oracle_bits(orc, a, s ^ t, m),
                          oracle_bits(orc, a, s, m) ^ oracle_bits(orc, a, t, m))


def test_toeplitz_is_diagonal_constant(orc):
    n, m = 40, 33
    s = rand_bits(n + m - 1, 61)
    cols = []
    for c in range(n):
        e = np.zeros(n, np.uint8)
        e[c] = 1
        cols.append(oracle_bits(orc, e, s, m, level=0))
    T = np.stack(cols, axis=1)                       # m x n
    assert np.array_equal(T[1:, 1:], T[:-1, :-1])    # T[r+1][c+1] = T[r][c]
    # every seed bit appears: first row and first column hold all n+m-1 bits
    assert T.shape == (m, n)


def test_toeplitz_edge_cases(orc):
    s = uniform_bits(200, 71)
    out = orc.toeplitz(np.zeros(1, np.uint64), 0, s, 200, 50)
    assert not out.any() and out.size == 1
    assert orc.toeplitz(uniform_bits(64, 1), 64, s, 200, 0).size == 0
    with pytest.raises(ValueError):
        orc.toeplitz(uniform_bits(100, 1), 100, s, 150, 60)  # needs 159 bits
    with pytest.raises(ValueError):
        orc.toeplitz(uniform_bits(10, 1), 10, s, 200, 20, cap=10)  # m > cap


def test_row_functions_agree_with_block(orc):
    n, m = 5000, 700
    x = uniform_bits(n, 81)
    s = uniform_bits(n + m - 1, 82)
    blk = unpack_bits(orc.toeplitz(x, n, s, n + m - 1, m), m)
    for r in (0, 1, 63, 64, 399, m - 1):
        assert orc.toeplitz_row(x, n, s, 0, m, r) == blk[r]
        assert orc.toeplitz_rowwin(x, n, s, n + m - 1, 0, m, r) == blk[r]


# ----------------------------------------------------------- concatenation ---

@pytest.mark.parametrize("stride_mode", ["shared", "independent"])
def test_hash_batch_concatenates_per_block_hashes(orc, stride_mode):
    n, ns = 20000, 9
    a = bernoulli_bits(n, 0.4, 91)
    sub, ln, wo, _ = orc.sample(a, n, ns, orc.SAMPLE_IID, key=92)
    m = orc.out_lengths(ln, orc.OUT_RATIO, 2, 5)
    cap = int(m.max())
    nmax = int(ln.max())
    stride = 0 if stride_mode == "shared" else nmax + cap - 1
    seed_bits = (ns - 1) * stride + nmax + cap - 1
    seed = uniform_bits(seed_bits, 93)
    out, total = orc.hash_batch(sub, ln, wo, m, seed, seed_bits, stride, cap,
                                level=1)
    assert total == int(m.sum())
    obits = unpack_bits(out, out.size * 64)
    sbits = unpack_bits(seed, seed_bits)
    off = 0
    for j in range(ns):
        nj, mj = int(ln[j]), int(m[j])
        xj = unpack_bits(sub[int(wo[j]):], nj)
        window = sbits[j * stride: j * stride + nj + cap - 1]
        want = toeplitz_by_fft(xj, window, mj, cap)
        assert np.array_equal(obits[off:off + mj], want), j
        off += mj
    assert not obits[total:].any()
    out0, _ = orc.hash_batch(sub, ln, wo, m, seed, seed_bits, stride, cap,
                             level=0)
    assert np.array_equal(out0, out)


# ---------------------------------------------------------- input helpers ---

def test_pack_roundtrip_and_tail():
    for n in (1, 63, 64, 65, 1000):
        b = rand_bits(n, n)
        w = pack_bits(b)
        assert w.size == (n + 63) // 64
        assert np.array_equal(unpack_bits(w, n), b)
        assert not unpack_bits(w, w.size * 64)[n:].any()


def test_bernoulli_density():
    n = 1 << 20
    for p in (0.2, 0.3, 0.5):
        frac = unpack_bits(bernoulli_bits(n, p, 5), n).mean()
        assert abs(frac - p) < 5 * np.sqrt(p * (1 - p) / n)


def test_toeplitz_ignores_input_bits_past_n(orc):
    # Bits beyond n in the last input word are not part of the input.
    for n, m in ((100, 40), (65, 65), (1000, 3)):
        x = uniform_bits(n, 101)
        dirty = x.copy()
        dirty[-1] |= ~np.uint64((1 << (n % 64)) - 1) if n % 64 else np.uint64(0)
        s = uniform_bits(n + m - 1, 102)
        for level in (0, 1):
            assert np.array_equal(orc.toeplitz(dirty, n, s, n + m - 1, m,
                                               level=level),
                                  orc.toeplitz(x, n, s, n + m - 1, m,
                                               level=level))
        for r in (0, m - 1):
            assert (orc.toeplitz_rowwin(dirty, n, s, n + m - 1, 0, m, r)
                    == orc.toeplitz_row(x, n, s, 0, m, r))


# ------------------------------------------------ sifting (Sec. III.B step 2)

@pytest.mark.parametrize("n,ns,pk", [(5000, 7, 0.6), (64 * 40, 3, 0.9),
                                     (1000, 1, 0.5), (777, 16, 0.0),
                                     (4096, 8, 1.0)])
def test_sift_equals_selection_by_v_and_keep(orc, n, ns, pk):
    """Sampling then sifting inside each sub-block == selecting, from the raw
    string, the rounds with V_i = j and keep_i = 1 (in ascending i)."""
    a = uniform_bits(n, n + 1)
    keep = bernoulli_bits(n, pk, n + 2) if 0.0 < pk < 1.0 else (
        uniform_bits(n, 1) & np.uint64(0) if pk == 0.0 else
        pack_bits(np.ones(n, dtype=np.uint8)))
    key = 0xABC + n
    sub, ln, wo, abort = orc.sample(a, n, ns, orc.SAMPLE_IID, key=key,
                                    keep=keep)
    v = orc.assign_iid(n, ns, key)
    abits, kbits = unpack_bits(a, n), unpack_bits(keep, n)
    assert int(ln.sum()) == int(kbits.sum())
    for j in range(ns):
        want = abits[(v == j) & (kbits == 1)]
        assert int(ln[j]) == want.size
        got = unpack_bits(sub[int(wo[j]):], int(ln[j])) if want.size else want
        assert np.array_equal(got, want), j


def test_sift_explicit_mode_and_permute_rejected(orc):
    n, ns = 3000, 5
    a = uniform_bits(n, 3)
    keep = bernoulli_bits(n, 0.7, 4)
    v = assignment(n, ns, 5)
    sub, ln, wo, _ = orc.sample(a, n, ns, orc.SAMPLE_EXPLICIT, assign=v,
                                keep=keep)
    abits, kbits = unpack_bits(a, n), unpack_bits(keep, n)
    for j in range(ns):
        want = abits[(v == j) & (kbits == 1)]
        assert np.array_equal(unpack_bits(sub[int(wo[j]):], int(ln[j])), want)
    with pytest.raises(ValueError):
        orc.sample(a, n, ns, orc.SAMPLE_PERMUTE, assign=permutation(n, 6),
                   keep=keep)


# ------------------------------------------- abort threshold (Sec. III.D) ---

def test_ub_tail_bounds_the_exact_binomial_tail(orc):
    """The Sec. III.D bound is an upper bound on P(Binomial(n, p) > L)."""
    from scipy.stats import binom
    for n in (100, 1000, 10 ** 5, 2 ** 28):
        for p in (1 / 2048, 0.01, 0.05, 0.3, 0.5):
            mu, sd = n * p, math.sqrt(n * p * (1 - p))
            for k in (0, 1, 2, 4, 7):
                L = int(math.ceil(mu + k * sd))
                if L >= n:
                    continue
                exact = float(binom.sf(L, n, p))
                bound = orc.ub_tail(n, p, L)
                assert exact <= bound * (1 + 1e-9) + 1e-300, (n, p, L)
                assert bound <= 1.0


def test_ub_tail_special_values(orc):
    assert orc.ub_tail(1000, 0.25, 250) == pytest.approx(0.5)   # H = 0
    assert orc.ub_tail(1000, 0.25, 1000) == 0.0                 # L = n
    assert orc.ub_tail(1000, 0.25, 100) == 1.0                  # below mean
    # Monotone: a larger threshold never has a larger bound.
    vals = [orc.ub_tail(10 ** 6, 0.01, L) for L in range(10000, 10600, 37)]
    assert all(b <= a for a, b in zip(vals, vals[1:]))


@pytest.mark.parametrize("n,p,ns,eps", [(2 ** 28, 1 / 2048, 2048, 1e-8),
                                        (2 ** 24, 0.3 / 128, 128, 1e-6),
                                        (10 ** 5, 0.05, 20, 1e-10),
                                        (200, 0.5, 2, 1e-30)])
def test_ub_threshold_is_the_smallest_valid_threshold(orc, n, p, ns, eps):
    from scipy.stats import binom
    L = orc.ub_threshold(n, p, ns, eps)
    assert ns * orc.ub_tail(n, p, L) <= eps
    if L > math.ceil(n * p):
        assert ns * orc.ub_tail(n, p, L - 1) > eps
    # The union bound with the exact tail holds as well.
    assert ns * float(binom.sf(L, n, p)) <= eps


# ------------------------------------------------ GEAT key length pins ---

GEAT_BASE = dict(n_rounds=1e9, p_x=0.02, q_tol=0.0082, eta_tol=1.0, e_bit=0.058,
                 f_ec=1.16, eps_sec=1e-6, eps_sm=1e-7, p_omega=1.0, d_x=3.0,
                 eps_abort=0.0, n_sub=1)


@pytest.mark.parametrize("eps", [1e-2, 1e-5, 1e-8, 1e-12, 1e-20])
def test_geat_g_matches_high_precision(orc, eps):
    """g(eps) = -log2(1 - sqrt(1 - eps^2)) (App. A) against an 80-digit
    decimal evaluation of that very expression."""
    from decimal import Decimal, getcontext
    getcontext().prec = 80
    e = Decimal(eps)
    val = -(1 - (1 - e * e).sqrt()).ln() / Decimal(2).ln()
    assert orc.geat_g(eps) == pytest.approx(float(val), rel=1e-13)


@pytest.mark.parametrize("q", [0.005, 0.0082, 0.05, 0.2])
def test_geat_tradeoff_is_tangent_below_the_entropy_bound(orc, q):
    """App. C: the affine min-tradeoff function is the tangent, at e_t, of
    the convex 1 - h2(e) at the tolerated error Q, so it never exceeds
    pZ^2 eta (1 - h2(Q)) and meets it exactly at e_t = Q."""
    p = dict(GEAT_BASE, q_tol=q, eta_tol=0.7)
    bound = (1 - p["p_x"]) ** 2 * 0.7 * (1 - (-q * math.log2(q)
                                              - (1 - q) * math.log2(1 - q)))
    assert orc.geat_terms(p, q)["h"] == pytest.approx(bound, rel=1e-14)
    for e in np.linspace(1e-4, 0.499, 200):
        assert orc.geat_terms(p, float(e))["h"] <= bound * (1 + 1e-14)
    assert orc.geat_terms(p, q * 0.9)["h"] < bound
    assert orc.geat_terms(p, min(0.49, q * 1.1))["h"] < bound


def test_geat_rate_tends_to_asymptotic_bbm92_rate(orc):
    """As N grows, the optimised key rate l/N tends to the asymptotic rate
    pZ^2 eta [1 - h2(Q) - f_EC h2(e_bit)] (the finite-size terms are
    o(N)), from below."""
    def h2(x):
        return -x * math.log2(x) - (1 - x) * math.log2(1 - x)
    p = dict(GEAT_BASE, eta_tol=0.9)
    asym = (1 - p["p_x"]) ** 2 * 0.9 * (1 - h2(p["q_tol"]) - p["f_ec"] * h2(p["e_bit"]))
    rates = []
    for n in [1e8, 1e10, 1e12, 1e16]:
        k, _, _ = orc.geat_optimise(dict(p, n_rounds=n))
        rates.append(k / n)
    assert all(r < asym for r in rates)
    assert all(b > a for a, b in zip(rates, rates[1:]))
    assert rates[-1] == pytest.approx(asym, rel=2e-3)


def test_geat_bound_is_at_least_eq1_of_sec_ii(orc):
    """Sec. II Eq. (1), H >= N h - v1 sqrt(N) - v0, is the App. A bound at
    one particular alpha, bounded from below with xi, beta(eps), gamma(eps);
    so the oracle's bound, maximised over alpha, can only be larger, and its
    sqrt(N) coefficient is at most v1 (tests/pin_checks.py)."""
    from tests.pin_checks import check_geat_eq1
    check_geat_eq1(orc.geat_key_length)


def test_geat_bound_has_the_closed_form_large_n_expansion(orc):
    """N h - max_alpha bound = c1 sqrt(N) + c0 + o(1) with the closed forms
    c1 = V sqrt(2 ln2 (g + L)) and c0 = g + 2L + 2 (g + L) K(0) / (ln2 V^2)
    derived from App. A in tests/pin_checks.py; this fixes the V^2 term, the
    squared (alpha - 1)/(2 - alpha) on K', d_X^2 inside V and the alpha
    log2(1/p_Omega) term."""
    from tests.pin_checks import check_geat_expansion
    check_geat_expansion(orc.geat_key_length)


def test_geat_diverges_at_both_ends_of_alpha(orc):
    """App. A: the (g + alpha log2(1/p_Omega)) / (alpha - 1) term blows up as
    alpha -> 1, K'(alpha) as alpha -> 3/2."""
    best, a, e = orc.geat_optimise(GEAT_BASE)
    assert best > 0 and 1 < a < 1.5 and 0 < e < 0.5
    assert orc.geat_key_length(GEAT_BASE, 1 + 1e-13, e) < -1e10
    assert orc.geat_key_length(GEAT_BASE, 1.5 - 1e-7, e) < -1e10


def test_geat_sub_block_loss_is_small_and_grows_with_n_sub(orc):
    """Claim 1 / Sec. IV: sampling into N_S sub-blocks costs key length,
    more for more sub-blocks, but only a little at N_S = 20 (p_S = 0.05)."""
    totals = []
    for ns in [1, 2, 5, 10, 20, 50]:
        p = dict(GEAT_BASE, n_sub=ns, eps_abort=1e-8 if ns > 1 else 0.0)
        totals.append(orc.geat_optimise(p)[0])
    assert all(b < a for a, b in zip(totals, totals[1:]))
    assert totals[4] > 0.9 * totals[0]
