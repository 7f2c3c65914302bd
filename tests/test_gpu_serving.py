"""Serving (continuous batching) on the GPU.

Each job is the whole method of Sec. III.B on one block: i.i.d. sampling with
the abort threshold, an independent seed window per sub-block drawn from the
job's seed key, the per-sub-block Toeplitz hash and the concatenation.  The
tests check results against the oracle, the same results alone and in a mix
(bit-exact: tolerance 0), admission under a small HBM budget, and errors.
"""

import math
import time

import numpy as np
import pytest

from tests.gpu_util import first_diff, to_dev, to_host
from workloads import bernoulli_bits

pytestmark = pytest.mark.gpu


def job_params(n, ns, l_ub, rule, a, b):
    """Sizes the library derives from a job (the rule stated in ssbh.h)."""
    mean = n / ns
    if not l_ub:
        l_ub = math.ceil(mean + 8.0 * math.sqrt(mean)) + 64
    n_cap = min(l_ub, n)
    m_cap = (n_cap * a) // b if rule == 1 else a
    stride = n_cap + (m_cap - 1 if m_cap else 0)
    return l_ub, n_cap, m_cap, stride, ns * stride


def oracle_job(orc, bits, n, ns, key, seed_key, rule, a, b, l_ub=0):
    l_ub, n_cap, m_cap, stride, seed_bits = job_params(n, ns, l_ub, rule, a, b)
    sub, ln, wo, abort = orc.sample(bits, n, ns, orc.SAMPLE_IID, key=key,
                                    l_ub=l_ub)
    if abort:
        return None, 0
    om = orc.out_lengths(ln, rule, a, b)
    seed = orc.seed_from_key(seed_key, seed_bits)
    return orc.hash_batch(sub, ln, wo, om, seed, seed_bits, stride, m_cap)


def wait(ctx, ids, timeout=120.0):
    res = {}
    t0 = time.time()
    while len(res) < len(ids):
        for i in ids:
            if i in res:
                continue
            r = ctx.poll(i)
            if r is not None:
                res[i] = r
        assert time.time() - t0 < timeout, "serving jobs did not finish"
        time.sleep(0.001)
    return res


JOBS = [  # (n_bits, n_sub, p, rule, a, b)
    (1 << 20, 16, 0.3, 1, 2, 5),
    ((1 << 18) + 12345, 5, 0.5, 1, 3, 10),
    (300000, 1, 0.2, 0, 777, 1),
    (1 << 21, 32, 0.4, 1, 1, 2),
    (123457, 7, 0.3, 0, 5000, 1),
    ((1 << 20) + 3, 64, 0.25, 1, 600, 1000),
]


@pytest.fixture(scope="module")
def inputs():
    return [bernoulli_bits(n, p, 1000 + k) for k, (n, _, p, *_r) in
            enumerate(JOBS)]


def test_jobs_match_oracle(orc, inputs):
    import torch
    from paper_2308_02856_amd import ssbh
    ctx = ssbh.Context(0, hbm_budget=1 << 30)
    devs = [to_dev(a) for a in inputs]
    torch.cuda.synchronize()
    made = []
    for k, (n, ns, p, rule, a, b) in enumerate(JOBS):
        job, out = ctx.make_job(devs[k], n, ns, 0x100 + k, 0x200 + k, rule,
                                a, b)
        made.append((ctx.submit(job), out, job))
    res = wait(ctx, [m[0] for m in made])
    for k, (jid, out, _) in enumerate(made):
        n, ns, p, rule, a, b = JOBS[k]
        r = res[jid]
        assert r.status == 0, (k, r.status)
        want, total = oracle_job(orc, inputs[k], n, ns, 0x100 + k, 0x200 + k,
                                 rule, a, b)
        assert r.out_bits == total
        got = to_host(out)[: want.size]
        assert np.array_equal(got, want), (k, first_diff(got, want))
    ctx.close()


def test_alone_equals_mix(inputs):
    """Every job's output is bit-identical when it runs alone and when it
    runs concurrently with all the others (tolerance: 0 differing bits)."""
    import torch
    from paper_2308_02856_amd import ssbh
    ctx = ssbh.Context(0, hbm_budget=1 << 30)
    devs = [to_dev(a) for a in inputs]
    torch.cuda.synchronize()
    specs = []
    for rep in range(3):
        for k, (n, ns, p, rule, a, b) in enumerate(JOBS):
            specs.append((k, n, ns, rule, a, b, 0x5000 + 17 * rep + k,
                          0x6000 + 31 * rep + k))
    alone = []
    for (k, n, ns, rule, a, b, key, skey) in specs:
        job, out = ctx.make_job(devs[k], n, ns, key, skey, rule, a, b)
        jid = ctx.submit(job)
        r = wait(ctx, [jid])[jid]
        assert r.status == 0
        alone.append(to_host(out).copy())
    made = []
    for (k, n, ns, rule, a, b, key, skey) in specs:
        job, out = ctx.make_job(devs[k], n, ns, key, skey, rule, a, b)
        made.append((ctx.submit(job), out))
    res = wait(ctx, [m[0] for m in made])
    overlapped = sum(1 for i in range(1, len(made))
                     if res[made[i][0]].t_admit < res[made[i - 1][0]].t_done)
    for i, (jid, out) in enumerate(made):
        assert res[jid].status == 0
        assert np.array_equal(to_host(out), alone[i]), i
    assert overlapped > 0, "no two jobs were on the device at the same time"
    ctx.close()


def test_small_budget_admits_in_turn(orc):
    """With a budget of 2.5 jobs, at most two jobs hold device memory at any
    time; all finish and match the oracle; a job larger than the budget is
    refused at submission."""
    import torch
    from paper_2308_02856_amd import ssbh
    n, ns = 1 << 21, 32
    bits = bernoulli_bits(n, 0.3, 9)
    dev = to_dev(bits)
    torch.cuda.synchronize()
    probe = ssbh.Context(0, hbm_budget=1 << 30)
    job, _ = probe.make_job(dev, n, ns, 1, 2, 1, 2, 5)
    jid = probe.submit(job)
    need = wait(probe, [jid])[jid].device_bytes
    probe.close()
    ctx = ssbh.Context(0, hbm_budget=int(2.5 * need))
    made = []
    for k in range(8):
        job, out = ctx.make_job(dev, n, ns, 0x900 + k, 0xA00 + k, 1, 2, 5)
        made.append((ctx.submit(job), out, k))
    res = wait(ctx, [m[0] for m in made])
    events = sorted([(r.t_admit, 1) for r in res.values()] +
                    [(r.t_done, -1) for r in res.values()])
    live = peak = 0
    for _, d in events:
        live += d
        peak = max(peak, live)
    assert peak <= 2
    for jid, out, k in made:
        want, total = oracle_job(orc, bits, n, ns, 0x900 + k, 0xA00 + k, 1, 2, 5)
        assert res[jid].status == 0 and res[jid].out_bits == total
        assert np.array_equal(to_host(out)[: want.size], want)
    # Two sub-blocks of 2^27 bits: the job's transforms alone (2^28 points)
    # are far beyond the budget (its content does not matter).
    big = torch.zeros(1 << 22, dtype=torch.int64, device="cuda")
    job, _ = ctx.make_job(big, 1 << 28, 2, 1, 2, 1, 2, 5)
    with pytest.raises(ssbh.SsbhError) as e:
        ctx.submit(job)
    assert e.value.status == ssbh.E_NOMEM
    ctx.close()


def test_abort_and_unknown_job(inputs):
    import torch
    from paper_2308_02856_amd import ssbh
    ctx = ssbh.Context(0, hbm_budget=1 << 28)
    n, ns = 1 << 20, 16
    dev = to_dev(inputs[0])
    torch.cuda.synchronize()
    job, _ = ctx.make_job(dev, n, ns, 0x77, 0x78, 1, 2, 5, l_ub=n // ns)
    jid = ctx.submit(job)
    r = wait(ctx, [jid])[jid]
    assert r.status == ssbh.E_ABORT_OVERSIZE
    with pytest.raises(ssbh.SsbhError):
        ctx.poll(jid)          # released after the terminal poll
    with pytest.raises(ssbh.SsbhError):
        ctx.poll(123456789)
    ctx.close()
