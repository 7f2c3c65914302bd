"""Bit-block, seed, permutation and assignment generators (numpy PCG64).

Layout shared by every part of the project: a bit string of ``n`` bits is a
``uint64`` array of ``ceil(n / 64)`` words; bit ``k`` is
``(w[k >> 6] >> (k & 63)) & 1`` (least significant bit first).  Bits past
``n`` in the last word are zero.
"""

from __future__ import annotations

import numpy as np

WORD_BITS = 64
_CHUNK = 1 << 24  # bits generated per numpy call, bounds temporary memory


def n_words(n_bits: int) -> int:
    return (int(n_bits) + WORD_BITS - 1) // WORD_BITS


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """Pack a 0/1 array into LSB-first uint64 words."""
    bits = np.asarray(bits, dtype=np.uint8).ravel()
    n = bits.size
    nw = n_words(n)
    padded = np.zeros(nw * WORD_BITS, dtype=np.uint8)
    padded[:n] = bits
    return np.packbits(padded, bitorder="little").view("<u8").astype(np.uint64)


def unpack_bits(words: np.ndarray, n_bits: int) -> np.ndarray:
    """Unpack LSB-first uint64 words into a 0/1 uint8 array of ``n_bits``."""
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
    out = np.unpackbits(w.view(np.uint8), bitorder="little")
    return out[: int(n_bits)]


def _tail_mask(words: np.ndarray, n_bits: int) -> np.ndarray:
    r = int(n_bits) % WORD_BITS
    if r and words.size:
        words[-1] &= np.uint64((1 << r) - 1)
    return words


def uniform_bits(n_bits: int, seed: int) -> np.ndarray:
    """``n_bits`` i.i.d. uniform bits (Bernoulli(1/2)), packed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nw = n_words(n_bits)
    words = rng.integers(0, np.iinfo(np.uint64).max, size=nw, dtype=np.uint64,
                         endpoint=True)
    return _tail_mask(words, n_bits)


def bernoulli_bits(n_bits: int, p: float, seed: int) -> np.ndarray:
    """``n_bits`` i.i.d. Bernoulli(p) bits, packed.

    ``p`` is realised as ``round(p * 65536) / 65536`` (each bit compares one
    uniform 16-bit draw against that threshold); ``p = 0.5`` takes the exact
    uniform-word path.
    """
    n_bits = int(n_bits)
    if abs(p - 0.5) < 1e-12:
        return uniform_bits(n_bits, seed)
    thr = int(round(p * 65536))
    rng = np.random.Generator(np.random.PCG64(seed))
    nw = n_words(n_bits)
    out = np.empty(nw, dtype=np.uint64)
    done = 0
    while done < n_bits:
        cnt = min(_CHUNK, n_bits - done)
        draws = rng.integers(0, 65536, size=cnt, dtype=np.uint16)
        bits = (draws < thr).astype(np.uint8)
        packed = pack_bits(bits)
        out[done // WORD_BITS: done // WORD_BITS + packed.size] = packed
        done += cnt
    return _tail_mask(out, n_bits)


def permutation(n: int, seed: int) -> np.ndarray:
    """A uniformly random permutation of ``0..n-1`` as uint32.

    numpy's ``Generator.shuffle`` is a Fisher-Yates shuffle driven by PCG64.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    pi = np.arange(int(n), dtype=np.uint32)
    rng.shuffle(pi)
    return pi


def assignment(n: int, n_sub: int, seed: int) -> np.ndarray:
    """Explicit sampling variables: ``n`` values uniform in ``[0, n_sub)``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, int(n_sub), size=int(n), dtype=np.uint32)
