"""Numerical check of the rounding bound behind complex-float storage in the
FFT hash (independent seeds, or one sub-block, transforms of at most 2^18
points).  The transform of z = s + i xr (seed window real, reversed input
bits imaginary) is taken in the library's four-step order -- 64-point DFTs
down the columns times w_L^(n2 k1), then row DFTs -- with the column stage's
output Y1 rounded to complex64, the spectrum squared, the inverse row DFTs and
inverse twiddles applied, that output Y2 rounded to complex64, and the
inverse column DFTs.  Half the imaginary part is s (*) xr.  The bound says
its error stays below 5 * 2^-24 * |z|^2 < 1/4 for L <= 2^18; this test
measures the error in double precision (numpy) against the exact integers and
checks the bound, for random and all-one inputs.  It checks the analysis,
not the GPU kernels (those are compared with the oracle bit for bit)."""

import numpy as np
import pytest

U = 2.0 ** -24


def four_step_joint(z: np.ndarray, round_f32: bool) -> np.ndarray:
    """c = z (*) z (cyclic, length L = 64 N2) by the four-step transform."""
    L = z.size
    n2 = L // 64
    a = z.reshape(64, n2)                       # a[n1, n2] = z[n1 N2 + n2]
    k1 = np.arange(64)[:, None]
    c2 = np.arange(n2)[None, :]
    tw = np.exp(-2j * np.pi * (k1 * c2) / L)
    y1 = np.fft.fft(a, axis=0) * tw             # columns, then twiddle
    if round_f32:
        y1 = y1.astype(np.complex64).astype(np.complex128)
    spec = np.fft.fft(y1, axis=1)               # rows
    y2 = np.fft.ifft(spec * spec, axis=1) * n2 * np.conj(tw)
    if round_f32:
        y2 = y2.astype(np.complex64).astype(np.complex128)
    c = np.fft.ifft(y2, axis=0) * 64 / L        # inverse columns, 1/L
    return c.reshape(L)


@pytest.mark.parametrize("L,n,m,ones", [(4096, 3000, 1000, False),
                                        (196608, 131072, 52428, False),
                                        (196608, 131072, 52428, True),
                                        (262144, 258049, 4096, True),
                                        (262144, 200000, 60000, False)])
def test_float_storage_error_within_bound(L, n, m, ones):
    rng = np.random.default_rng(L + n)
    if ones:
        s = np.ones(L)
        x = np.ones(n)
    else:
        s = rng.integers(0, 2, L).astype(np.float64)
        x = (rng.random(n) < 0.3).astype(np.float64)
    xr = np.zeros(L)
    xr[:n] = x[::-1]
    z = s + 1j * xr
    exact = np.rint(four_step_joint(z, False).imag / 2.0)
    approx = four_step_joint(z, True).imag / 2.0
    err = np.max(np.abs(approx - exact))
    norm2 = float(np.sum(s) + np.sum(x))          # |z|^2: the ones of s and x
    bound = 5.0 * U * norm2
    assert norm2 <= L + n
    assert err <= bound, (err, bound)
    assert bound < 0.25
    # The entries the hash reads round to the middle product itself.
    q = np.arange(n - 1, n + m - 1)
    mp = np.convolve(s[: n + m - 1], xr[:n])[q] if L <= 4096 else None
    if mp is not None:
        assert np.array_equal(np.rint(approx[q]), mp)


def test_bound_fails_past_the_limit():
    """Above 2^18 points the same bound no longer stays below 1/4 for every
    input, which is why longer transforms keep doubles."""
    L = 1 << 19
    assert 5.0 * U * (2 * L) > 0.25
    assert 5.0 * U * (2 * (1 << 18)) < 0.25
