"""The five workloads of this project and the serving job stream.

Each workload is described by plain numbers; the keys are fixed so that every
run (tests, benchmark, smoke check) sees the same synthetic data.

* ``small``       N = 2^18 uniform bits, keyed Fisher-Yates permutation
                  (Durstenfeld, SplitMix64 stream of perm_key) then a
                  contiguous split into 8 sub-blocks of 2^15 bits, each hashed
                  to 2^14 bits with its own seed of 2^15 + 2^14 - 1 bits.
* ``single``      one block, n = 2^24 uniform bits hashed to m = 2^23 bits
                  with a seed of n + m - 1 bits (no sampling).
* ``batched``     N = 2^28 Bernoulli(0.3) bits, i.i.d. uniform assignment to
                  2048 sub-blocks, output floor(0.4 * n_j) bits each, one
                  shared seed of max n_j + max m_j - 1 bits (or, as the
                  paper's protocol has it, an independent seed window per
                  sub-block at stride max n_j + max m_j - 1).
* ``contraction`` N = 2^30 uniform bits, keyed permutation then split into 8192
                  sub-blocks of 2^17 bits, shared seed, 2^16 output bits each.
* ``serving``     a Poisson stream (mean 200 jobs/s) of jobs with block sizes
                  log-uniform in 2^20..2^28, Bernoulli(p), p ~ U[0.2, 0.5]
                  realised per job as round(p 2^10)/2^10 (serving_input),
                  sub-block size log-uniform in 2^16..2^18, output ratio
                  q/1000 with q uniform in 200..600, fresh keys per job.
* ``TABLE1``      the five input/output sizes of the paper's FPGA experiment
                  (96.04 .. 1920 Mbit in, 6.054 .. 152.56 Mbit out), uniform
                  bits, hashed as one block and by 20 sub-blocks.
"""

from __future__ import annotations

import math

import numpy as np

from .gen import uniform_bits

_KEY_BASE = 0x2308028560000000

CONFIGS = {
    "small": dict(
        name="small", n_bits=1 << 18, p=0.5, n_sub=8, sampling="permute",
        out_rule="fixed", out_a=1 << 14, out_b=1,
        seed_mode="independent", sub_bits=1 << 15,
        input_seed=1, perm_key=_KEY_BASE + 0x101, seed_seed=201,
    ),
    "single": dict(
        name="single", n_bits=1 << 24, p=0.5, n_sub=1, sampling="none",
        out_rule="fixed", out_a=1 << 23, out_b=1, seed_mode="shared",
        input_seed=2, seed_seed=202,
    ),
    "batched": dict(
        name="batched", n_bits=1 << 28, p=0.3, n_sub=2048, sampling="iid",
        out_rule="ratio", out_a=2, out_b=5, seed_mode="shared",
        input_seed=3, sample_key=_KEY_BASE + 0x103, seed_seed=203,
        indep_seed_seed=303,   # independent seeds: stride n_max + m_max - 1
    ),
    "contraction": dict(
        name="contraction", n_bits=1 << 30, p=0.5, n_sub=8192,
        sampling="permute", out_rule="fixed", out_a=1 << 16, out_b=1,
        seed_mode="shared", sub_bits=1 << 17,
        input_seed=4, perm_key=_KEY_BASE + 0x104, seed_seed=204,
    ),
    "serving": dict(
        name="serving", rate_hz=200.0, log2_n=(20, 28), p=(0.2, 0.5),
        log2_sub=(16, 18), q=(200, 600), stream_seed=5,
        sample_key_base=_KEY_BASE + 0x105, seed_key_base=_KEY_BASE + 0x205,
    ),
}


# Table I of the paper (Sec. IV.C): input and output sizes of the FPGA
# experiment (Mbit) and its measured speeds in output bits per second, for
# direct hashing of one block ("traditional"; not measured at the two largest
# sizes) and for the sub-block method with p_S = 0.05, i.e. 20 sub-blocks.
# Context only: other hardware.
TABLE1 = [
    dict(input_mbit=96.040, output_mbit=6.054, fpga_traditional=498.60,
         fpga_ours=9899.80),
    dict(input_mbit=192.08, output_mbit=13.302, fpga_traditional=249.31,
         fpga_ours=4972.47),
    dict(input_mbit=288.12, output_mbit=20.736, fpga_traditional=166.24,
         fpga_ours=3318.63),
    dict(input_mbit=960.40, output_mbit=74.406, fpga_traditional=None,
         fpga_ours=997.05),
    dict(input_mbit=1920.00, output_mbit=152.56, fpga_traditional=None,
         fpga_ours=498.62),
]
TABLE1_N_SUB = 20


def table1_instance(k: int) -> dict:
    """Sizes and keys of Table I row k: n input bits (uniform), m output
    bits in total; the sub-block method divides the input i.i.d. into
    TABLE1_N_SUB sub-blocks and gives each floor(m / TABLE1_N_SUB) output
    bits, hashed with its own seed."""
    row = TABLE1[k]
    n = int(round(row["input_mbit"] * 1e6))
    m = int(round(row["output_mbit"] * 1e6))
    return dict(row, n_bits=n, m_bits=m, n_sub=TABLE1_N_SUB,
                sub_out=m // TABLE1_N_SUB, input_seed=1000 + k,
                seed_seed=2000 + k, sub_seed_seed=3000 + k,
                sample_key=_KEY_BASE + 0x110 + k)


def config(name: str) -> dict:
    return dict(CONFIGS[name])


def serving_jobs(count: int, seed: int = 5, rate_hz: float = 200.0,
                 log2_n=(20, 28), log2_sub=(16, 18), q=(200, 600),
                 p=(0.2, 0.5), max_n_bits: int | None = None) -> list[dict]:
    """A reproducible Poisson job stream.

    Every job carries its arrival time (seconds from stream start), its block
    size, Bernoulli parameter, sub-block count, output ratio ``q/1000`` and
    two fresh 64-bit keys (sampling variables and Toeplitz seed).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    jobs = []
    for k in range(int(count)):
        t += float(rng.exponential(1.0 / rate_hz))
        u = float(rng.random())
        n_bits = int(math.floor(2.0 ** (log2_n[0] + (log2_n[1] - log2_n[0]) * u)))
        if max_n_bits is not None:
            n_bits = min(n_bits, int(max_n_bits))
        us = float(rng.random())
        sub = int(math.floor(2.0 ** (log2_sub[0] + (log2_sub[1] - log2_sub[0]) * us)))
        n_sub = max(1, int(round(n_bits / sub)))
        qq = int(rng.integers(q[0], q[1] + 1))
        pp = float(p[0] + (p[1] - p[0]) * rng.random())
        jobs.append(dict(
            index=k, arrival_s=t, n_bits=n_bits, p=pp, n_sub=n_sub,
            ratio_num=qq, ratio_den=1000,
            sample_key=int(rng.integers(0, 2**63 - 1)) * 2 + 1,
            seed_key=int(rng.integers(0, 2**63 - 1)) * 2 + 1,
        ))
    return jobs


SERVING_P_BITS = 10      # a job's p is realised as round(p * 2^10) / 2^10
SERVING_POOL_BITS = 1 << 28


def serving_planes(seed: int = 55, pool_bits: int = SERVING_POOL_BITS,
                   planes: int = SERVING_P_BITS) -> list[np.ndarray]:
    """Independent uniform bit pools (numpy PCG64), one per binary digit of
    the serving jobs' Bernoulli threshold."""
    return [uniform_bits(pool_bits, seed + k) for k in range(planes)]


def _serving_layout(job: dict, pool_words: int) -> tuple[int, int, int]:
    """(word offset, words, threshold) of one job's input."""
    nw = (job["n_bits"] + 63) // 64
    off = (job["index"] * 7919) % max(1, pool_words - nw + 1)
    thr = int(round(job["p"] * (1 << SERVING_P_BITS)))
    return off, nw, thr


def _below_threshold(planes, thr: int, ones, inv):
    """Bits of [U < thr] word-parallel, U's binary digits taken from the
    planes, most significant first (a comparator over bit slices).  `ones`
    is an all-one word array, `inv` bitwise complement."""
    lt = ones & 0
    eq = ones
    for b, x in enumerate(planes):
        if (thr >> (SERVING_P_BITS - 1 - b)) & 1:
            lt = lt | (eq & inv(x))
            eq = eq & x
        else:
            eq = eq & inv(x)
    return lt


def serving_input(job: dict, planes: list[np.ndarray]) -> np.ndarray:
    """The packed input of one serving job: n_bits i.i.d. Bernoulli(thr/2^10)
    bits, thr = round(p 2^10), bit i = [U_i < thr] where the 10 binary digits
    of U_i are bit i of a job-specific word slice of each plane pool."""
    off, nw, thr = _serving_layout(job, planes[0].size)
    sl = [pl[off: off + nw] for pl in planes]
    ones = np.full(nw, np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    words = _below_threshold(sl, thr, ones, np.invert).astype(np.uint64)
    r = job["n_bits"] % 64
    if r:
        words[-1] &= np.uint64((1 << r) - 1)
    return words


def serving_input_device(job: dict, d_planes: list):
    """serving_input computed with torch on the planes' device copies
    (int64 tensors holding the same words); bit-identical to the host."""
    import torch
    off, nw, thr = _serving_layout(job, d_planes[0].numel())
    sl = [pl[off: off + nw] for pl in d_planes]
    ones = torch.full((nw,), -1, dtype=torch.int64, device=d_planes[0].device)
    words = _below_threshold(sl, thr, ones, torch.bitwise_not)
    r = job["n_bits"] % 64
    if r:
        words[-1] &= (1 << r) - 1
    return words
