"""GPU: whole outputs of the benchmark workloads against the oracle.

tests/golden/make_digests.py runs the CPU oracle (only) on the benchmark's
exact inputs and stores the SHA-256 of each whole output.  Here the library
computes the same workloads with every kernel and schedule the benchmark's
tuner can pick, and the SHA-256 of each whole output must match (bit-exact,
tolerance 0): the single block (2^24 -> 2^23), the batched workload (2^28
bits, 2048 uneven sub-blocks) and the contraction workload (2^30 bits, keyed
permutation, 8192 x 2^17 -> 2^16).
"""

import hashlib
import json
import os

import numpy as np
import pytest

from tests.gpu_util import to_dev, to_host
from workloads import bernoulli_bits, config, uniform_bits

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def reference(workload: str) -> dict:
    """The oracle's digest of a workload (tests/golden/make_digests.py)."""
    with open(os.path.join(HERE, "golden", "digests.json")) as fh:
        return json.load(fh)[workload]


# The tuner's candidates (csrc/tune.hip): VALU (r, waves, chunk columns),
# matrix cores (mt, nt, wm, K split), FFT chunks of 64..256 MiB of transforms.
VALU = [(16, 4, 4096), (32, 2, 2048), (32, 4, 2048), (16, 8, 2048), (16, 2, 1024)]
MFMA = [(8, 2, 4, 0), (8, 2, 4, 1), (4, 2, 4, 0), (8, 1, 4, 0), (4, 4, 4, 0)]
FFT_MIB = [64, 128, 160, 192, 256]


def digest(t, bits: int) -> str:
    nw = (int(bits) + 63) // 64
    w = np.ascontiguousarray(to_host(t)[:nw])
    return hashlib.sha256(w.astype("<u8").tobytes()).hexdigest()


def fft_chunks(seed_bits: int, m_cap: int, point_bytes: int = 16):
    """Transform counts of the tuner's FFT chunk sizes at this seed length:
    L = the smallest 2^k or 3 * 2^k >= seed_bits (4096 <= L; 6144 is not
    used), 16 bytes per point (8 where the passes exchange floats)."""
    lengths = sorted(v for k in range(12, 32) for v in (1 << k, 3 << k)
                     if v != 6144)
    L = next(v for v in lengths if v >= max(seed_bits, 4096))
    return sorted({max(1, (mib << 20) // (point_bytes * L)) for mib in FFT_MIB})


def run_all(ctx, hash_, seed_bits, cap, want, bits, with_valu=True):
    """Hash with every candidate schedule; every digest equals `want`."""
    from paper_2308_02856_amd import ssbh
    seen = []
    for cp in fft_chunks(seed_bits, cap):
        ctx.set_fft_schedule(cp)
        seen.append((f"fft:{cp}", digest(hash_(ssbh.K_FFT), bits)))
    ctx.set_fft_schedule(0)
    for mt, nt, wm, ks in MFMA:
        ctx.set_mfma_schedule(mt, nt, wm, ks)
        seen.append((f"mfma:{mt}:{nt}:{wm}:{ks}",
                     digest(hash_(ssbh.K_MFMA_I8), bits)))
    ctx.set_mfma_schedule(0, 0, 0, 0)
    if with_valu:
        for r, w, cc in VALU:
            ctx.set_schedule(r, w, 0, cc)
            seen.append((f"valu:{r}:{w}:{cc}", digest(hash_(ssbh.K_VALU), bits)))
        ctx.set_schedule(0, 0, 0, 0)
    bad = [name for name, d in seen if d != want]
    assert not bad, bad


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02856_amd import ssbh
    c = ssbh.Context(0)
    yield c
    c.close()


def test_single_block_whole_output(ctx):
    import torch
    from paper_2308_02856_amd import ssbh
    ref = reference("single")
    c = config("single")
    n, m = c["n_bits"], c["out_a"]
    x = to_dev(uniform_bits(n, c["input_seed"]))
    seed_bits = n + m - 1
    seed = to_dev(uniform_bits(seed_bits, c["seed_seed"]))
    ln = torch.tensor([n], dtype=torch.int64, device="cuda")
    wo = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.empty((m + 63) // 64, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    for kern in (ssbh.K_FFT, ssbh.K_VALU):
        out.fill_(-1)
        _, tot, _ = ctx.hash_batch(x, x.numel(), ln, wo, 1, seed, seed_bits, m,
                                   out_rule=ssbh.OUT_FIXED, out_a=m, out=out,
                                   out_capacity_bits=m, status=st, kernel=kern)
        torch.cuda.synchronize()
        assert int(st.item()) == 0 and int(tot.item()) == ref["bits"] == m
        assert digest(out, m) == ref["sha256"], kern


def test_batched_whole_output(ctx):
    """Sub-block buffer and output of the batched step, every schedule."""
    import torch
    from paper_2308_02856_amd import ssbh
    ref = reference("batched")
    c = config("batched")
    n, ns, key = c["n_bits"], c["n_sub"], c["sample_key"]
    l_ub, _ = ssbh.ub_threshold(n, 1.0 / ns, ns, 1e-8)
    assert l_ub == ref["l_ub"]
    d_in = to_dev(bernoulli_bits(n, c["p"], c["input_seed"]))
    sub, ln, wo, st = ctx.sample(d_in, n, ns, ssbh.SAMPLE_IID, key=key,
                                 l_ub=l_ub)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    lens = to_host(ln)[:ns].astype(np.int64)
    woff = to_host(wo)[:ns].astype(np.int64)
    used = int(woff[-1] + (lens[-1] + 63) // 64)
    assert digest(sub, 64 * used) == ref["sub_sha256"]
    mlen = lens * c["out_a"] // c["out_b"]
    cap = int(mlen.max())
    seed_bits = int(lens.max()) + cap - 1
    assert seed_bits == ref["seed_bits"]
    seed = to_dev(uniform_bits(seed_bits, c["seed_seed"]))
    out_cap = int(mlen.sum())
    assert out_cap == ref["bits"]
    out = torch.empty((out_cap + 63) // 64, dtype=torch.int64, device="cuda")

    def hash_(kern):
        out.fill_(-1)
        _, tot, s = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed,
                                   seed_bits, cap, out_rule=ssbh.OUT_RATIO,
                                   out_a=c["out_a"], out_b=c["out_b"], out=out,
                                   out_capacity_bits=out_cap, kernel=kern)
        torch.cuda.synchronize()
        assert int(s.item()) == 0 and int(tot.item()) == out_cap
        return out

    run_all(ctx, hash_, seed_bits, cap, ref["sha256"], out_cap)
    # The library's own choice (autotuned) as well.
    ctx.tune(sub, sub.numel(), ln, wo, ns, seed, seed_bits, cap,
             out_rule=ssbh.OUT_RATIO, out_a=c["out_a"], out_b=c["out_b"],
             out=out, out_capacity_bits=out_cap)
    assert digest(hash_(ssbh.K_AUTO), out_cap) == ref["sha256"]


def test_batched_independent_whole_output(ctx):
    """The batched workload with the paper's independent seeds (stride
    max n_j + max m_j - 1): the FFT at every chunk size the tuner tries
    (floats between the passes, the library's choice at this length, and
    doubles) and the VALU kernel give the oracle's whole output."""
    import torch
    from paper_2308_02856_amd import ssbh
    ref = reference("batched_independent")
    c = config("batched")
    n, ns, key = c["n_bits"], c["n_sub"], c["sample_key"]
    l_ub, _ = ssbh.ub_threshold(n, 1.0 / ns, ns, 1e-8)
    d_in = to_dev(bernoulli_bits(n, c["p"], c["input_seed"]))
    sub, ln, wo, st = ctx.sample(d_in, n, ns, ssbh.SAMPLE_IID, key=key,
                                 l_ub=l_ub)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    lens = to_host(ln)[:ns].astype(np.int64)
    mlen = lens * c["out_a"] // c["out_b"]
    cap = int(mlen.max())
    stride = int(lens.max()) + cap - 1
    seed_bits = ns * stride
    assert stride == ref["stride"] and seed_bits == ref["seed_bits"]
    seed = to_dev(uniform_bits(seed_bits, c["indep_seed_seed"]))
    out_cap = int(mlen.sum())
    assert out_cap == ref["bits"]
    out = torch.empty((out_cap + 63) // 64, dtype=torch.int64, device="cuda")

    def hash_(kern):
        out.fill_(-1)
        _, tot, s = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed,
                                   seed_bits, cap, out_rule=ssbh.OUT_RATIO,
                                   out_a=c["out_a"], out_b=c["out_b"], out=out,
                                   out_capacity_bits=out_cap, seed_stride=stride,
                                   kernel=kern)
        torch.cuda.synchronize()
        assert int(s.item()) == 0 and int(tot.item()) == out_cap
        return out

    bad = []
    for bits, pb in ((0, 8), (64, 16)):
        ctx.set_fft_storage(bits)
        try:
            for cp in fft_chunks(stride, cap, pb):
                ctx.set_fft_schedule(cp)
                if digest(hash_(ssbh.K_FFT), out_cap) != ref["sha256"]:
                    bad.append(f"fft:{cp}:storage{bits}")
        finally:
            ctx.set_fft_schedule(0)
            ctx.set_fft_storage(0)
    if digest(hash_(ssbh.K_VALU), out_cap) != ref["sha256"]:
        bad.append("valu")
    assert not bad, bad


def test_contraction_whole_output(ctx):
    """Keyed permutation (its SHA-256 too), gather, then every matrix-core,
    FFT and bit-sliced schedule and the fp4 variant."""
    import torch
    from paper_2308_02856_amd import ssbh
    ref = reference("contraction")
    c = config("contraction")
    n, ns, L, m = c["n_bits"], c["n_sub"], c["sub_bits"], c["out_a"]
    perm = ctx.permutation(c["perm_key"], n)
    torch.cuda.synchronize()
    ph = hashlib.sha256(perm.cpu().numpy().view(np.uint32).astype("<u4")
                        .tobytes()).hexdigest()
    assert ph == ref["perm_sha256"]
    d_in = to_dev(uniform_bits(n, c["input_seed"]))
    sub, ln, wo, st = ctx.sample(d_in, n, ns, ssbh.SAMPLE_PERMUTE,
                                 assign=perm)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    del perm, d_in
    seed_bits = L + m - 1
    seed = to_dev(uniform_bits(seed_bits, c["seed_seed"]))
    out = torch.empty(ns * m // 64, dtype=torch.int64, device="cuda")

    def hash_(kern):
        out.fill_(-1)
        _, tot, s = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed,
                                   seed_bits, m, out_rule=ssbh.OUT_FIXED,
                                   out_a=m, out=out, out_capacity_bits=ns * m,
                                   kernel=kern)
        torch.cuda.synchronize()
        assert int(s.item()) == 0 and int(tot.item()) == ns * m
        return out

    run_all(ctx, hash_, seed_bits, m, ref["sha256"], ns * m, with_valu=False)
    ctx.set_schedule(16, 4, 0, 4096)
    assert digest(hash_(ssbh.K_VALU), ns * m) == ref["sha256"]
    ctx.set_schedule(0, 0, 0, 0)
    assert digest(hash_(ssbh.K_MFMA_F4), ns * m) == ref["sha256"]
