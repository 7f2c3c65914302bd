"""GPU: ssbh_hash_batch_noalloc, the variant of ssbh_hash_batch that
allocates nothing (plan, tiles and counters in the library's fixed device
array), against ssbh_hash_batch on the same arguments: bit-exact, on two calls
in a row with the second input smaller, and with every kernel it supports."""

import numpy as np
import pytest

from tests.gpu_util import to_dev
from workloads import bernoulli_bits, uniform_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02856_amd import ssbh
    c = ssbh.Context(0)
    yield c
    c.close()


def sampled(ctx, n, ns, key, p=0.4):
    import torch
    from paper_2308_02856_amd import ssbh
    a = bernoulli_bits(n, p, n % 991)
    sub, ln, wo, st = ctx.sample(to_dev(a), n, ns, ssbh.SAMPLE_IID, key=key)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    lens = ln.cpu().numpy()[:ns]
    return sub, ln, wo, lens


def both(ctx, sub, ln, wo, ns, lens, kernel, stride_mode):
    """(reference output, no-alloc output, totals) for one request."""
    import torch
    from paper_2308_02856_amd import ssbh
    mlen = lens * 2 // 5
    cap = int(max(1, mlen.max()))
    nmax = int(max(1, lens.max()))
    stride = nmax + cap - 1 if stride_mode else 0
    seed_bits = (ns - 1) * stride + nmax + cap - 1
    seed = to_dev(uniform_bits(seed_bits, 77 + ns))
    out_cap = int(mlen.sum())
    ref, rtot, rst = ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed,
                                    seed_bits, cap, out_rule=ssbh.OUT_RATIO,
                                    out_a=2, out_b=5, seed_stride=stride,
                                    kernel=ssbh.K_VALU)
    out = torch.full((max(1, (out_cap + 63) // 64),), -1, dtype=torch.int64,
                     device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.hash_batch_noalloc(sub, sub.numel(), ln, wo, ns, seed, seed_bits, cap,
                           out, out_cap, tot, st, out_rule=ssbh.OUT_RATIO,
                           out_a=2, out_b=5, seed_stride=stride, kernel=kernel)
    torch.cuda.synchronize()
    assert int(rst.item()) == 0 and int(st.item()) == 0
    assert int(tot.item()) == int(rtot.item()) == out_cap
    nw = (out_cap + 63) // 64
    return ref[:nw], out[:nw]


@pytest.mark.parametrize("kernel_name", ["valu", "mfma", "mfma_f4", "auto"])
def test_noalloc_equals_hash_batch_twice(ctx, kernel_name):
    """A large call, then a smaller one reusing the same fixed array."""
    import torch
    from paper_2308_02856_amd import ssbh
    kernel = {"valu": ssbh.K_VALU, "mfma": ssbh.K_MFMA_I8,
              "mfma_f4": ssbh.K_MFMA_F4, "auto": ssbh.K_AUTO}[kernel_name]
    for n, ns in (((1 << 21) + 77, 128), ((1 << 17) + 5, 64)):
        sub, ln, wo, lens = sampled(ctx, n, ns, 0x900 + ns)
        ref, got = both(ctx, sub, ln, wo, ns, lens, kernel, False)
        assert torch.equal(ref, got), (kernel_name, n, ns)


def test_noalloc_independent_seeds_twice(ctx):
    """Independent seeds (VALU), a large call then a smaller one."""
    import torch
    from paper_2308_02856_amd import ssbh
    for n, ns in (((1 << 20) + 3, 40), (70001, 3)):
        sub, ln, wo, lens = sampled(ctx, n, ns, 0xA00 + ns)
        ref, got = both(ctx, sub, ln, wo, ns, lens, ssbh.K_VALU, True)
        assert torch.equal(ref, got), (n, ns)


def test_noalloc_refuses_what_does_not_fit(ctx):
    """Errors come back before anything is enqueued: the FFT kernel, and a
    tile list larger than the fixed array; the output stays untouched."""
    import torch
    from paper_2308_02856_amd import ssbh
    ns = 16384
    ln = torch.full((ns,), 1 << 20, dtype=torch.int64, device="cuda")
    wo = torch.zeros(ns, dtype=torch.int64, device="cuda")
    sub = torch.zeros(1 << 10, dtype=torch.int64, device="cuda")
    seed = torch.zeros(1 << 10, dtype=torch.int64, device="cuda")
    out = torch.full((8,), 5, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    for kernel in (ssbh.K_FFT, ssbh.K_VALU):
        with pytest.raises(ssbh.SsbhError) as e:
            ctx.hash_batch_noalloc(sub, 1 << 30, ln, wo, ns, seed, 1 << 16,
                                   1 << 24, out, 512, tot, st,
                                   out_rule=ssbh.OUT_FIXED, out_a=1 << 24,
                                   kernel=kernel)
        assert e.value.status == ssbh.E_UNSUPPORTED
    torch.cuda.synchronize()
    assert out.tolist() == [5] * 8 and int(st.item()) == 0
