#!/usr/bin/env python3
"""Benchmark of the sampled sub-block hashing hot path on one MI355X.

One step = the whole hot path on the batched workload: i.i.d. sampling of
N = 2^28 Bernoulli(0.3) bits into 2048 sub-blocks (with the abort check),
then the Toeplitz hash of every sub-block (floor(0.4 n_j) output bits, one
shared seed of max n_j + max m_j - 1 bits) and the concatenation.  `value` is
input Gbit/s of that step with the input resident in HBM.  The same line
reports the plain single-block hash (n = 2^24 -> m = 2^23) that the method is
compared with (bit-sliced kernel and FFT, the faster one counts), the contraction workload (2^30 bits, 8192 equal sub-blocks,
int8 matrix cores against the bit-sliced kernel), the small workload through a
captured HIP graph, the five input/output sizes of the paper's Table I (one
block and 20 sub-blocks with independent seeds, both by the FFT hash), the serving stream (p50/p99 latency, sustained Gbit/s),
rooflines (the hash's row pass per launch, timed with HIP events on its
stream; the whole FFT hash; the sampling kernels against HBM), the rate of a
plain 1 GiB device copy beside the published HBM peak, and the CPU oracle
timed on a bounded sample.  The step's largest kernel is the sampling scatter
(0.64 ms); its roofline entry shows how far below HBM its LDS work keeps it.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("input Gbit/s hashed, batched sub-block vs plain single-block; "
          "p50/p99 latency")
CLOCK_GHZ = 2.4          # MI355X peak engine clock
LANES_PER_CU_CLK = 128   # 32-bit VALU lanes retired per CU per clock
BITOPS_PER_LANE_OP = 32  # v_bitop3_b32: 32 AND-XOR bit-products per lane
INT8_PEAK_TOPS = 5000.0  # MI355X dense int8 matrix peak (TOP/s)
FP4_PEAK_TFLOPS = 10100.0  # MI355X dense fp4 matrix peak (TFLOP/s)
HBM_PEAK_GBS = 8000.0    # MI355X HBM3E peak (GB/s)

KERNEL_SOURCES = {"k_toeplitz_valu": "hash_valu.hip",
                  "k_toeplitz_mfma": "hash_mfma.hip",
                  "k_fft_rows": "hash_fft.hip"}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")


def to_host(t):
    return t.detach().cpu().numpy().view(np.uint64)


def alu_peak_tbitops(num_cus: int) -> float:
    """256 CUs x 128 lanes x 2.4 GHz = 78.6 T 32-bit lane-ops/s (the FP32
    vector peak of 157.3 TFLOP/s counts an FMA as 2); one v_bitop3_b32 lane-op
    is 32 AND-XOR bit-products."""
    return num_cus * LANES_PER_CU_CLK * CLOCK_GHZ * 1e9 * BITOPS_PER_LANE_OP / 1e12


def kernel_source_digest(kernel: str) -> str:
    """Digest of the source file that holds the kernel's body."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2308_02856_amd", "csrc",
                           KERNEL_SOURCES[kernel]), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str, schedule: str):
    """HBM bytes per launch from committed PMC counters, if they were taken
    on the same kernel source and schedule (one record per schedule the
    tuner may pick)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            data = json.load(fh)
        rec = data.get(f"{kernel}:{workload}:{schedule}")
        if not rec or rec.get("source_digest") != kernel_source_digest(kernel):
            return None
        if rec.get("schedule") != schedule:
            return None
        return rec.get("hbm_bytes_per_launch")
    except (OSError, ValueError):
        return None


def kernel_avgs(rep: dict) -> dict:
    return {k: round(ms * 1e3 / n, 2) for k, (n, ms) in rep.items()}


DIGESTS = os.path.join(ROOT, "tests", "golden", "digests.json")


def load_digests() -> dict:
    """SHA-256 digests of the oracle's whole outputs on the benchmark's
    inputs, written by tests/golden/make_digests.py (oracle only)."""
    try:
        with open(DIGESTS) as fh:
            return json.load(fh)
    except OSError:
        return {}


def words_digest(words: np.ndarray, bits: int) -> str:
    nw = (int(bits) + 63) // 64
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64)[:nw])
    return hashlib.sha256(w.astype("<u8").tobytes()).hexdigest()


def time_events(fn, reps: int) -> list[float]:
    """Milliseconds of each call of fn, from HIP events on the current stream."""
    import torch
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        out.append(e0.elapsed_time(e1))
    return out


def run_batched(ctx, ssbh, args):
    import torch
    from workloads import bernoulli_bits, config, uniform_bits
    c = config("batched")
    n, ns, key = c["n_bits"], c["n_sub"], c["sample_key"]
    log(f"batched: generating {n} Bernoulli({c['p']}) input bits")
    a = bernoulli_bits(n, c["p"], c["input_seed"])
    d_in = to_dev(a)
    sub, ln, wo, st = ctx.sample(d_in, n, ns, ssbh.SAMPLE_IID, key=key)
    torch.cuda.synchronize()
    lens = to_host(ln)[:ns].astype(np.int64)
    mlen = lens * c["out_a"] // c["out_b"]
    cap = int(mlen.max())
    seed_bits = int(lens.max()) + cap - 1
    seed = to_dev(uniform_bits(seed_bits, c["seed_seed"]))
    # Abort threshold from the Sec. III.D tail bound: every round is kept,
    # so a sub-block's length is Binomial(N, 1/N_S); abort chance <= 1e-8.
    l_ub, _ = ssbh.ub_threshold(n, 1.0 / ns, ns, 1e-8)
    sub_cap = sub.numel()
    out_cap = int(mlen.sum())
    out = torch.empty((out_cap + 63) // 64, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    work = int((lens * mlen).sum())
    kernel = {"auto": ssbh.K_AUTO, "valu": ssbh.K_VALU,
              "mfma": ssbh.K_MFMA_I8, "fft": ssbh.K_FFT}[args.kernel]
    tune_report = ""
    if args.fft_chunk:
        ctx.set_fft_schedule(args.fft_chunk)
    if kernel == ssbh.K_AUTO and not args.no_tune:
        log("batched: autotuning the hash kernel (untimed)")
        tune_report = ctx.tune(sub, sub_cap, ln, wo, ns, seed, seed_bits, cap,
                               out_rule=ssbh.OUT_RATIO, out_a=c["out_a"],
                               out_b=c["out_b"], out=out,
                               out_capacity_bits=out_cap, total=tot, status=st,
                               reps=5)

    def sample():
        ctx.sample(d_in, n, ns, ssbh.SAMPLE_IID, key=key, l_ub=l_ub, sub=sub,
                   sub_capacity=sub_cap, length=ln, word_off=wo, status=st)

    def hash_():
        ctx.hash_batch(sub, sub_cap, ln, wo, ns, seed, seed_bits, cap,
                       out_rule=ssbh.OUT_RATIO, out_a=c["out_a"],
                       out_b=c["out_b"], out=out, out_capacity_bits=out_cap,
                       total=tot, status=st, reset_status=False, kernel=kernel)

    for _ in range(args.warmup):
        sample()
        hash_()
    torch.cuda.synchronize()
    log(f"batched: timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sample()
        hash_()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    status = int(st.item())
    if status != 0:
        raise RuntimeError(f"device status {ssbh.status_name(status)}")
    ms_step = (t1 - t0) * 1e3 / args.steps
    hash_ms = time_events(hash_, max(3, args.steps))
    schedule = ctx.last_schedule()
    samp_ms = time_events(sample, max(3, args.steps))
    # Per-kernel durations from the library's HIP events on the launch
    # stream: the FFT passes' launches record their own start and end
    # (hipExtLaunchKernelGGL), the other kernels are bracketed by events.
    ctx.set_timing(True)
    reps = max(3, args.steps)
    for _ in range(reps):
        hash_()
    hash_kernels = ctx.timing_report()
    for _ in range(reps):
        sample()
    sample_kernels = ctx.timing_report()
    ctx.set_timing(False)
    # Sampling with sifting flags (Sec. III.B step 2): 96 % of rounds kept.
    keep = to_dev(bernoulli_bits(n, 0.96, c["input_seed"] + 1000))
    sub2 = torch.empty_like(sub)
    ln2, wo2 = torch.empty_like(ln), torch.empty_like(wo)
    st2 = torch.zeros_like(st)
    l_ub2, _ = ssbh.ub_threshold(n, 0.96 / ns, ns, 1e-8)

    def sample_sifted():
        ctx.sample_sifted(d_in, keep, n, ns, ssbh.SAMPLE_IID, key=key,
                          l_ub=l_ub2, sub=sub2, sub_capacity=sub_cap,
                          length=ln2, word_off=wo2, status=st2)

    sample_sifted()
    sift_ms = time_events(sample_sifted, 3)
    if int(st2.item()) != 0:
        raise RuntimeError("sifted sampling status nonzero")
    del keep, sub2
    res = dict(n=n, ns=ns, lens=lens, mlen=mlen, cap=cap, seed_bits=seed_bits,
               work=work, ms_step=ms_step,
               hash_ms=float(np.mean(hash_ms)), sample_ms=float(np.mean(samp_ms)),
               a=a, out=out, sub=sub, ln=ln, wo=wo, st=st, seed=seed, key=key,
               c=c, sample=sample,
               schedule=schedule, tune_report=tune_report, l_ub=l_ub,
               hash_kernels=hash_kernels, sample_kernels=sample_kernels,
               timed_calls=reps,
               sift_ms=float(np.mean(sift_ms)), l_ub_sifted=l_ub2)
    return res


def fft_schedule_parts(schedule: str):
    """(transform length, sub-blocks per transform, bytes per transform
    point between passes) of an FFT schedule name "fft:<chunk>:x<per>:L<L>"
    with ":f32" appended when the passes exchange complex floats."""
    L = int(schedule.split(":L")[1].split(":")[0])
    per = int(schedule.split(":x")[1].split(":")[0])
    return L, per, (8 if schedule.endswith(":f32") else 16)


def fft_hash_roofline(schedule: str, ns: int, n_bits: int, out_bits: int,
                      hash_ms: float, shared: bool, launches: int) -> dict:
    """The whole FFT hash (all passes, two chunks in flight) against HBM.
    Algorithmic bytes per hash: every transform is written by the column
    pass, read and written by the row pass and read by the output pass
    (4 L points of 16 bytes, or of 8 with float storage); with a shared
    seed the spectrum is built once (48 L) and read by every row-pass launch
    (16 L each); the packed input bits are read once and the output bits are
    written twice and read once (parity words, then their places)."""
    L, per, pb = fft_schedule_parts(schedule)
    transforms = (ns + per - 1) // per
    b = 4 * pb * L * transforms + n_bits // 8 + 3 * out_bits // 8
    if shared:
        b += 48 * L + 16 * L * launches
    achieved = b / (hash_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernels": "k_fft_cols + k_fft_rows + k_fft_out "
            "+ k_fft_emit (+ spectrum)", "schedule": schedule,
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "algorithmic_bytes_per_hash": int(b), "hash_ms": round(hash_ms, 4)}


def copy_rate_gbps(mib: int = 1024, reps: int = 3) -> float:
    """Read + write bytes per second of a plain device copy of `mib` MiB
    (HIP events): the rate a streaming kernel reaches on this HBM, reported
    beside the published peak the roofline fractions use."""
    import torch
    a = torch.ones((mib << 20) // 8, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ms = float(np.mean(time_events(lambda: b.copy_(a), reps)))
    del a, b
    torch.cuda.empty_cache()
    return 2 * (mib << 20) / (ms * 1e-3) / 1e9


def sampling_roofline(res) -> dict:
    """Sampling (a1-a3) against HBM: per call it must read the N input
    bits once and write the N bits of the sub-block buffer once (2 N / 8
    bytes); its two kernels' HIP-event time per call is the denominator.
    The kernels are bound by their LDS work (match tables, cursors and the
    image, with bank conflicts on random addresses) and by the SplitMix64
    draws made in both passes, not by HBM; the fraction shows how far."""
    sk = res["sample_kernels"]
    calls = res["timed_calls"]
    us = {k: ms * 1e3 / calls for k, (n_l, ms) in sk.items()}
    t_s = sum(us.values()) * 1e-6
    bytes_call = 2 * res["n"] // 8
    achieved = bytes_call / t_s / 1e9
    return {"bound": "hbm", "kernels": sorted(sk), "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "algorithmic_bytes_per_call": bytes_call,
            "us_per_call": round(t_s * 1e6, 2),
            "limit": "LDS (profiles/lds_counters__sampling_batched_2p28_2048sub.txt)"}


def run_batched_independent(ctx, ssbh, args, res):
    """The batched step with the paper's independent seeds (Sec. III.B
    step 3): sub-block j hashed with its own seed window at stride
    S = max n_j + max m_j - 1 (seed of 2048 S bits).  The tuner picks among
    the FFT (one transform per sub-block: seed window real, bits imaginary,
    spectrum squared) at each chunk size and the VALU schedules."""
    import torch
    from workloads import uniform_bits
    c, ns, lens, mlen, cap = res["c"], res["ns"], res["lens"], res["mlen"], res["cap"]
    sub, ln, wo, st = res["sub"], res["ln"], res["wo"], res["st"]
    stride = int(lens.max()) + cap - 1
    seed_bits = ns * stride
    seed = to_dev(uniform_bits(seed_bits, c["indep_seed_seed"]))
    out_cap = int(mlen.sum())
    out = torch.empty((out_cap + 63) // 64, dtype=torch.int64, device="cuda")
    outv = torch.empty_like(out)
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")

    def hash_(kern, o):
        ctx.hash_batch(sub, sub.numel(), ln, wo, ns, seed, seed_bits, cap,
                       out_rule=ssbh.OUT_RATIO, out_a=c["out_a"],
                       out_b=c["out_b"], out=o, out_capacity_bits=out_cap,
                       total=tot, status=st, reset_status=False,
                       seed_stride=stride, kernel=kern)

    kern = ssbh.K_AUTO
    tune_report = ""
    if args.no_tune:
        kern = ssbh.K_FFT              # chunk from --fft-chunk (else default)
    else:
        log("batched, independent seeds: autotuning (untimed)")
        tune_report = ctx.tune(sub, sub.numel(), ln, wo, ns, seed, seed_bits,
                               cap, out_rule=ssbh.OUT_RATIO, out_a=c["out_a"],
                               out_b=c["out_b"], seed_stride=stride, out=out,
                               out_capacity_bits=out_cap, total=tot, status=st,
                               reps=5)
    hash_(kern, out)
    hash_(ssbh.K_VALU, outv)
    torch.cuda.synchronize()
    if int(st.item()) != 0:
        raise RuntimeError("independent-seed hash: device status nonzero")
    same = bool(torch.equal(out, outv))
    hash_ms = float(np.mean(time_events(lambda: hash_(kern, out),
                                        max(3, args.steps))))
    hash_(kern, out)
    schedule = ctx.last_schedule()
    valu_ms = float(np.mean(time_events(lambda: hash_(ssbh.K_VALU, outv), 2)))
    # The same hash with complex doubles between the FFT passes (the
    # library keeps floats there at this length): time and equality.
    ctx.set_fft_storage(64)
    try:
        hash_(ssbh.K_FFT, outv)
        f64_ms = float(np.mean(time_events(lambda: hash_(ssbh.K_FFT, outv), 3)))
        f64_schedule = ctx.last_schedule()
    finally:
        ctx.set_fft_storage(0)
    torch.cuda.synchronize()
    f64_equal = bool(torch.equal(out, outv)) and int(st.item()) == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res["sample"]()
        hash_(kern, out)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    if int(st.item()) != 0:
        raise RuntimeError("independent-seed step: device status nonzero")
    oracle_equal = digest_equal("batched_independent", out, out_cap)
    item = {"workload": "batched_independent", "seed_stride": stride,
            "seed_bits": seed_bits, "hash_kernel": schedule,
            "ms_per_step": round(ms_step, 4),
            "gbps_step": round(res["n"] / (ms_step * 1e-3) / 1e9, 3),
            "hash_ms": round(hash_ms, 4), "hash_ms_valu": round(valu_ms, 4),
            "hash_ms_fft_f64_storage": round(f64_ms, 4),
            "fft_f64_storage_schedule": f64_schedule,
            "fft_f64_storage_equal": f64_equal,
            "gbps_hash": round(res["n"] / (hash_ms * 1e-3) / 1e9, 3),
            "auto_equals_valu": same, "oracle_digest_equal": oracle_equal,
            "tuning": tune_report.strip().splitlines()}
    if schedule.startswith("fft"):
        # Row pass in the joint mode: each transform is read and written
        # once (L complex points each way, doubles or floats); there is no
        # seed spectrum.
        ctx.set_timing(True)
        reps = max(3, args.steps)
        for _ in range(reps):
            hash_(kern, out)
        hk = ctx.timing_report()
        ctx.set_timing(False)
        n_l, ms = hk["k_fft_rows"]
        L, _, pb = fft_schedule_parts(schedule)
        total_bytes = reps * ns * 2 * L * pb
        achieved = total_bytes / (ms * 1e-3) / 1e9
        item["roofline"] = {
            "bound": "hbm", "kernel": "k_fft_rows", "schedule": schedule,
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": load_traffic("k_fft_rows", "batched_independent",
                                    schedule),
            "avg_launch_us": round(ms * 1e3 / n_l, 2),
            "algorithmic_bytes_per_launch": int(total_bytes / n_l)}
        item["kernel_avg_us"] = kernel_avgs(hk)
        item["roofline_hash"] = fft_hash_roofline(schedule, ns, res["n"],
                                                  out_cap, hash_ms, False, 0)
    del seed, out, outv
    torch.cuda.empty_cache()
    return item


def run_single(ctx, ssbh, args):
    import torch
    from workloads import config, uniform_bits
    c = config("single")
    n, m = c["n_bits"], c["out_a"]
    x = to_dev(uniform_bits(n, c["input_seed"]))
    seed_bits = n + m - 1
    seed = to_dev(uniform_bits(seed_bits, c["seed_seed"]))
    ln = torch.tensor([n], dtype=torch.int64, device="cuda")
    wo = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.empty((m + 63) // 64, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")

    def hash_(kernel):
        ctx.hash_batch(x, x.numel(), ln, wo, 1, seed, seed_bits, m,
                       out_rule=ssbh.OUT_FIXED, out_a=m, out=out,
                       out_capacity_bits=m, total=tot, status=st,
                       reset_status=False, kernel=kernel)

    res = dict(n=n, m=m, work=n * m)
    words = {}
    for name, kern in (("valu", ssbh.K_VALU), ("fft", ssbh.K_FFT)):
        hash_(kern)
        torch.cuda.synchronize()
        log(f"single: timing {args.single_steps} {name} hashes of {n} -> {m} bits")
        ms = time_events(lambda: hash_(kern), args.single_steps)
        if int(st.item()) != 0:
            raise RuntimeError(f"single-block device status nonzero ({name})")
        res[f"ms_{name}"] = float(np.mean(ms))
        words[name] = out.clone()
    res["fft_equals_valu"] = bool(torch.equal(words["valu"], words["fft"]))
    res["ms"] = min(res["ms_valu"], res["ms_fft"])
    res["oracle_digest_equal"] = digest_equal("single", words["fft"], m)
    return res


def digest_equal(workload: str, out, bits: int):
    """The whole output against the oracle's SHA-256 of it (None when the
    digest file has no entry for the workload)."""
    ref = load_digests().get(workload)
    if not ref:
        return None
    return (int(bits) == ref["bits"] and
            words_digest(to_host(out), bits) == ref["sha256"])


# ------------------------------------------------------------------ Table I

def run_table1(ctx, ssbh, args):
    """The input/output sizes of the paper's FPGA experiment (Table I, five
    rows, uniform synthetic bits), hashed on the GPU two ways with the FFT
    hash: one block directly ("traditional", seed n + m - 1 bits) and the
    sub-block method (i.i.d. division into 20 sub-blocks, floor(m / 20)
    output bits each, every sub-block with its own seed of L_S^UB + l - 1
    bits, L_S^UB at eps = 1e-8).  Speeds are output bits per second, the unit
    of the table, next to the FPGA's (context: other hardware).  The first
    row is also hashed by the bit-sliced kernel and must give the same bits."""
    import torch
    from workloads import TABLE1, table1_instance, uniform_bits
    out_rows = []
    ks = range(len(TABLE1)) if args.table1_rows is None else [
        int(v) for v in args.table1_rows.split(",")]
    for k in ks:
        c = table1_instance(k)
        n, m, ns, lt = c["n_bits"], c["m_bits"], c["n_sub"], c["sub_out"]
        log(f"table1 row {k}: {n} -> {m} bits")
        x = to_dev(uniform_bits(n, c["input_seed"]))
        # Traditional: one block.
        sb = n + m - 1
        seed = to_dev(uniform_bits(sb, c["seed_seed"]))
        ln = torch.tensor([n], dtype=torch.int64, device="cuda")
        wo = torch.zeros(1, dtype=torch.int64, device="cuda")
        out = torch.empty((m + 63) // 64, dtype=torch.int64, device="cuda")
        tot = torch.zeros(1, dtype=torch.int64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")

        def trad(kernel=ssbh.K_FFT):
            ctx.hash_batch(x, x.numel(), ln, wo, 1, seed, sb, m,
                           out_rule=ssbh.OUT_FIXED, out_a=m, out=out,
                           out_capacity_bits=m, total=tot, status=st,
                           reset_status=False, kernel=kernel)

        trad()
        torch.cuda.synchronize()
        ms_trad = float(np.mean(time_events(trad, args.table1_reps)))
        if int(st.item()) != 0:
            raise RuntimeError(f"table1 row {k}: traditional status {int(st.item())}")
        trad_sched = ctx.last_schedule()
        row = {"input_mbit": c["input_mbit"], "output_mbit": c["output_mbit"],
               "traditional": {"ms": round(ms_trad, 3),
                               "out_bits_per_s": round(m / (ms_trad * 1e-3)),
                               "in_gbps": round(n / (ms_trad * 1e-3) / 1e9, 3),
                               "schedule": trad_sched}}
        if k == 0:
            ref = out.clone()
            trad(ssbh.K_VALU)
            torch.cuda.synchronize()
            row["traditional"]["fft_equals_valu"] = bool(
                int(st.item()) == 0 and torch.equal(ref, out))
        del seed
        # Sub-block method: 20 sub-blocks, independent seeds.
        l_ub, _ = ssbh.ub_threshold(n, 1.0 / ns, ns, 1e-8)
        S = l_ub + lt - 1
        seeds = to_dev(uniform_bits(ns * S, c["sub_seed_seed"]))
        subcap = (n + 63) // 64 + ns
        sub = torch.empty(subcap, dtype=torch.int64, device="cuda")
        lens = torch.empty(ns, dtype=torch.int64, device="cuda")
        woffs = torch.empty(ns, dtype=torch.int64, device="cuda")
        sst = torch.zeros(1, dtype=torch.int32, device="cuda")
        o2 = torch.empty((ns * lt + 63) // 64, dtype=torch.int64, device="cuda")
        tot2 = torch.zeros(1, dtype=torch.int64, device="cuda")
        st2 = torch.zeros(1, dtype=torch.int32, device="cuda")

        def sample():
            ctx.sample(x, n, ns, ssbh.SAMPLE_IID, key=c["sample_key"], l_ub=l_ub,
                       sub=sub, sub_capacity=subcap, length=lens, word_off=woffs,
                       status=sst)

        def ours(kernel=ssbh.K_FFT):
            sample()
            ctx.hash_batch(sub, subcap, lens, woffs, ns, seeds, ns * S, lt,
                           out_rule=ssbh.OUT_FIXED, out_a=lt, seed_stride=S,
                           out=o2, out_capacity_bits=ns * lt, total=tot2,
                           status=st2, reset_status=False, kernel=kernel)

        ours()
        torch.cuda.synchronize()
        ms_ours = float(np.mean(time_events(ours, args.table1_reps)))
        ms_samp = float(np.mean(time_events(sample, args.table1_reps)))
        if int(sst.item()) != 0 or int(st2.item()) != 0:
            raise RuntimeError(f"table1 row {k}: status {int(sst.item())}/"
                               f"{int(st2.item())}")
        row["ours"] = {"ms": round(ms_ours, 3), "sample_ms": round(ms_samp, 3),
                       "out_bits_per_s": round(ns * lt / (ms_ours * 1e-3)),
                       "in_gbps": round(n / (ms_ours * 1e-3) / 1e9, 3),
                       "n_sub": ns, "sub_out_bits": lt, "l_ub": l_ub,
                       "seed_stride": S, "schedule": ctx.last_schedule()}
        if k == 0:
            ref = o2.clone()
            ours(ssbh.K_VALU)
            torch.cuda.synchronize()
            row["ours"]["fft_equals_valu"] = bool(
                int(st2.item()) == 0 and torch.equal(ref, o2))
        row["fpga_out_bits_per_s"] = {"traditional": c["fpga_traditional"],
                                      "ours": c["fpga_ours"]}
        row["gpu_ours_over_fpga_ours"] = round(
            row["ours"]["out_bits_per_s"] / c["fpga_ours"])
        row["ours_over_traditional_gpu"] = round(ms_trad / ms_ours, 2)
        out_rows.append(row)
        del x, seeds, sub, out, o2
        torch.cuda.empty_cache()
    return {"workload": "table1", "speed_unit": "output bits/s",
            "kernel": "fft", "data": "uniform synthetic bits", "rows": out_rows}


# -------------------------------------------------------------- contraction

def run_contraction(ctx, ssbh, args, peak_alu):
    """2^30 uniform bits, permutation split into 8192 sub-blocks of 2^17 bits,
    2^16 output bits each from one shared seed: the gather, then the hash on
    the int8 matrix cores and on the bit-sliced VALU kernel (same bits)."""
    import torch
    from workloads import config, uniform_bits
    c = config("contraction")
    n, ns, L, m = c["n_bits"], c["n_sub"], c["sub_bits"], c["out_a"]
    log(f"contraction: {n} bits, permutation split into {ns} x {L}")
    d_in = to_dev(uniform_bits(n, c["input_seed"]))
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    perm_ms = float(np.mean(time_events(
        lambda: ctx.permutation(c["perm_key"], n, out=perm), 2)))
    seed_bits = L + m - 1
    seed = to_dev(uniform_bits(seed_bits, c["seed_seed"]))
    sub_cap = ns * (L // 64)
    sub = torch.empty(sub_cap, dtype=torch.int64, device="cuda")
    ln = torch.empty(ns, dtype=torch.int64, device="cuda")
    wo = torch.empty(ns, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.empty(ns * m // 64, dtype=torch.int64, device="cuda")
    outv = torch.empty_like(out)
    outf = torch.empty_like(out)
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")

    def sample():
        ctx.sample(d_in, n, ns, ssbh.SAMPLE_PERMUTE, assign=perm, sub=sub,
                   sub_capacity=sub_cap, length=ln, word_off=wo, status=st)

    def hash_(kern, o):
        ctx.hash_batch(sub, sub_cap, ln, wo, ns, seed, seed_bits, m,
                       out_rule=ssbh.OUT_FIXED, out_a=m, out=o,
                       out_capacity_bits=ns * m, total=tot, status=st,
                       reset_status=False, kernel=kern)

    out4 = torch.empty_like(out)
    sample()
    hash_(ssbh.K_MFMA_I8, out)
    hash_(ssbh.K_VALU, outv)
    hash_(ssbh.K_FFT, outf)
    hash_(ssbh.K_MFMA_F4, out4)
    torch.cuda.synchronize()
    same = bool(torch.equal(out, outv)) and int(st.item()) == 0
    same_fft = bool(torch.equal(out, outf))
    same_f4 = bool(torch.equal(out, out4))
    oracle_equal = digest_equal("contraction", out, ns * m)
    g_ms = float(np.mean(time_events(sample, 3)))
    # Per-kernel times of the streaming gather, and the direct gather (one
    # random input-word read per output bit) on the same permutation.
    ctx.set_timing(True)
    for _ in range(3):
        sample()
    gather_kernels = kernel_avgs(ctx.timing_report())
    ctx.set_timing(False)
    ctx.set_sample_path(1)
    sub_direct = torch.empty_like(sub)
    ctx.sample(d_in, n, ns, ssbh.SAMPLE_PERMUTE, assign=perm, sub=sub_direct,
               sub_capacity=sub_cap, length=ln, word_off=wo, status=st)
    gd_ms = float(np.mean(time_events(
        lambda: ctx.sample(d_in, n, ns, ssbh.SAMPLE_PERMUTE, assign=perm,
                           sub=sub_direct, sub_capacity=sub_cap, length=ln,
                           word_off=wo, status=st), 2)))
    ctx.set_sample_path(0)
    torch.cuda.synchronize()
    gather_equal = bool(torch.equal(sub, sub_direct)) and int(st.item()) == 0
    # The same split through the context's keyed permutation of perm_key:
    # the first call builds it and buckets it, later calls with that key
    # keep both and run the window and merge passes only.
    def sample_keyed():
        ctx.sample(d_in, n, ns, ssbh.SAMPLE_PERMUTE, key=c["perm_key"],
                   sub=sub_direct, sub_capacity=sub_cap, length=ln,
                   word_off=wo, status=st)
    sample_keyed()
    gk_ms = float(np.mean(time_events(sample_keyed, 3)))
    torch.cuda.synchronize()
    gather_keyed_equal = bool(torch.equal(sub, sub_direct)) and int(st.item()) == 0
    del sub_direct
    mf_ms = float(np.mean(time_events(lambda: hash_(ssbh.K_MFMA_I8, out), 3)))
    mfma_sched = ctx.last_schedule()
    f4_ms = float(np.mean(time_events(lambda: hash_(ssbh.K_MFMA_F4, out4), 3)))
    va_ms = float(np.mean(time_events(lambda: hash_(ssbh.K_VALU, outv), 2)))
    ff_ms = float(np.mean(time_events(lambda: hash_(ssbh.K_FFT, outf), 3)))
    prods = L * m * ns
    del d_in, perm, sub, out, outv, outf, out4
    torch.cuda.empty_cache()
    return {
        "workload": "contraction", "n_bits": n, "n_sub": ns, "sub_bits": L,
        "m_bits": m, "permutation_ms": round(perm_ms, 3),
        "gather_ms": round(g_ms, 3),
        "gather_kernel_avg_us": gather_kernels,
        "gather_direct_ms": round(gd_ms, 3),
        "gather_equals_direct": gather_equal,
        "gather_keyed_ms": round(gk_ms, 3),
        "gather_keyed_equal": gather_keyed_equal,
        "gbps_step_fft_keyed": round(n / ((gk_ms + ff_ms) * 1e-3) / 1e9, 3),
        "mfma_ms": round(mf_ms, 3), "valu_ms": round(va_ms, 3),
        "gbps_step_mfma": round(n / ((g_ms + mf_ms) * 1e-3) / 1e9, 3),
        "gbps_hash_mfma": round(n / (mf_ms * 1e-3) / 1e9, 3),
        "gbps_hash_valu": round(n / (va_ms * 1e-3) / 1e9, 3),
        "mfma_int8_tops": round(2 * prods / (mf_ms * 1e-3) / 1e12, 1),
        "mfma_frac": round(2 * prods / (mf_ms * 1e-3) / 1e12 / INT8_PEAK_TOPS, 4),
        "valu_frac": round(prods / (va_ms * 1e-3) / 1e12 / peak_alu, 4),
        "fft_ms": round(ff_ms, 3),
        "gbps_step_fft": round(n / ((g_ms + ff_ms) * 1e-3) / 1e9, 3),
        "gbps_hash_fft": round(n / (ff_ms * 1e-3) / 1e9, 3),
        "mfma_f4_ms": round(f4_ms, 3),
        "mfma_f4_tops": round(2 * prods / (f4_ms * 1e-3) / 1e12, 1),
        "mfma_f4_frac": round(2 * prods / (f4_ms * 1e-3) / 1e12 / FP4_PEAK_TFLOPS, 4),
        "mfma_equals_valu": same,
        "fft_equals_mfma": same_fft,
        "mfma_f4_equals_int8": same_f4,
        "oracle_digest_equal": oracle_equal,
        "mfma_traffic": load_traffic("k_toeplitz_mfma", "contraction",
                                     mfma_sched),
    }


def run_gather(ctx, ssbh, args):
    """Permutation sampling of the contraction workload alone (the keyed
    permutation of 2^30 entries built once, then `steps` gathers), for
    profiler passes over the gather kernels."""
    import torch
    from workloads import config, uniform_bits
    c = config("contraction")
    n, ns = c["n_bits"], c["n_sub"]
    d_in = to_dev(uniform_bits(n, c["input_seed"]))
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.permutation(c["perm_key"], n, out=perm)
    sub = torch.empty(n // 64, dtype=torch.int64, device="cuda")
    ln = torch.empty(ns, dtype=torch.int64, device="cuda")
    wo = torch.empty(ns, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")

    def sample():
        ctx.sample(d_in, n, ns, ssbh.SAMPLE_PERMUTE, assign=perm, sub=sub,
                   sub_capacity=n // 64, length=ln, word_off=wo, status=st)

    ms = time_events(sample, max(1, args.steps))
    torch.cuda.synchronize()
    return {"mode": "gather", "n_bits": n, "n_sub": ns,
            "gather_ms": round(float(np.mean(ms)), 3),
            "status": int(st.item())}


# -------------------------------------------------------------------- small

def run_small(ctx, ssbh, args):
    """The small workload (2^18 bits, permutation split into 8 x 2^15 bits,
    2^14 output bits each from independent seeds): eager calls against one
    replay of the captured HIP graph, per pass."""
    import torch
    from workloads import config, uniform_bits
    c = config("small")
    n, ns, L, m = c["n_bits"], c["n_sub"], c["sub_bits"], c["out_a"]
    stride = L + m - 1
    seed_bits = ns * stride
    d_in = to_dev(uniform_bits(n, c["input_seed"]))
    perm = ctx.permutation(c["perm_key"], n)
    seed = to_dev(uniform_bits(seed_bits, c["seed_seed"]))
    sub_cap = ns * (L // 64)
    sub = torch.empty(sub_cap, dtype=torch.int64, device="cuda")
    ln = torch.empty(ns, dtype=torch.int64, device="cuda")
    wo = torch.empty(ns, dtype=torch.int64, device="cuda")
    out = torch.empty(ns * m // 64, dtype=torch.int64, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")

    def eager():
        ctx.sample(d_in, n, ns, ssbh.SAMPLE_PERMUTE, assign=perm, sub=sub,
                   sub_capacity=sub_cap, length=ln, word_off=wo, status=st)
        ctx.hash_batch(sub, sub_cap, ln, wo, ns, seed, seed_bits, m,
                       out_rule=ssbh.OUT_FIXED, out_a=m, out=out,
                       out_capacity_bits=ns * m, total=tot, status=st,
                       reset_status=False, seed_stride=stride,
                       kernel=ssbh.K_VALU)

    pipe = ctx.pipeline(d_in=d_in, n_bits=n, n_sub=ns,
                        mode=ssbh.SAMPLE_PERMUTE, d_assign=perm, d_sub=sub,
                        sub_capacity_words=sub_cap, d_len=ln, d_word_off=wo,
                        out_rule=ssbh.OUT_FIXED, out_a=m, out_b=1, d_seed=seed,
                        seed_bits=seed_bits, seed_stride=stride, m_cap=m,
                        kernel=ssbh.K_VALU, d_out=out,
                        out_capacity_bits=ns * m, d_out_total_bits=tot,
                        d_status=st)
    eager()
    torch.cuda.synchronize()
    ref = out.clone()
    pipe.launch()
    torch.cuda.synchronize()
    same = bool(torch.equal(out, ref)) and int(st.item()) == 0
    reps = 200

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    e_ms = timed(eager)
    g_ms = timed(pipe.launch)
    # One replay at a time on an idle stream, bracketed by HIP events: the
    # device's latency per pass (the back-to-back figure above is bound by
    # the host's graph submissions).
    dev_ms = float(np.median(time_events(pipe.launch, 50)))
    pipe.close()
    return {"workload": "small", "n_bits": n, "n_sub": ns,
            "eager_ms": round(e_ms, 4), "graph_ms": round(g_ms, 4),
            "graph_device_ms": round(dev_ms, 4),
            "gbps_graph": round(n / (g_ms * 1e-3) / 1e9, 3),
            "graph_equals_eager": same}


# ------------------------------------------------------------------ serving

def run_serving(ssbh, args):
    """Poisson stream of whole-method jobs (i.i.d. sampling with the abort
    threshold, independent seeds from the job's key, hash, concatenation),
    admitted FIFO under an HBM budget; latency = submit -> results ready."""
    import torch
    from workloads import (CONFIGS, serving_input_device, serving_jobs,
                           serving_planes)
    cfg = CONFIGS["serving"]
    total = args.serve_jobs + args.serve_warmup
    jobs = serving_jobs(total, seed=cfg["stream_seed"], rate_hz=cfg["rate_hz"],
                        log2_n=cfg["log2_n"], log2_sub=cfg["log2_sub"],
                        q=cfg["q"], p=cfg["p"])
    log(f"serving: {total} job inputs, each Bernoulli(p) with its own p")
    d_planes = [to_dev(pl) for pl in serving_planes()]
    ctx = ssbh.Context(0, hbm_budget=args.serve_budget_mib << 20)
    made = []
    for jb in jobs:
        d_in = serving_input_device(jb, d_planes)
        job, out = ctx.make_job(d_in, jb["n_bits"], jb["n_sub"],
                                jb["sample_key"], jb["seed_key"],
                                ssbh.OUT_RATIO, jb["ratio_num"],
                                jb["ratio_den"])
        made.append((jb, job, out, d_in))
    del d_planes
    torch.cuda.synchronize()
    ids = [None] * len(made)
    log(f"serving: submitting {total} jobs at {cfg['rate_hz']:.0f}/s")
    t_start = time.perf_counter()

    def submitter():
        for i, (jb, job, _, _) in enumerate(made):
            delay = t_start + jb["arrival_s"] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            ids[i] = ctx.submit(job)

    th = threading.Thread(target=submitter)
    th.start()
    results = {}
    nxt = 0
    pending = []
    deadline = time.perf_counter() + jobs[-1]["arrival_s"] + 120.0
    while len(results) < len(made):
        while nxt < len(made) and ids[nxt] is not None:
            pending.append(nxt)
            nxt += 1
        still = []
        for i in pending:
            r = ctx.poll(ids[i])
            if r is None:
                still.append(i)
            else:
                results[i] = r
        pending = still
        if time.perf_counter() > deadline:
            raise RuntimeError("serving stream did not drain")
        time.sleep(0.0005)
    th.join()
    ctx.close()
    checked, equal = serving_digest_check(made, results)
    meas = range(args.serve_warmup, len(made))
    lat = np.array([(results[i].t_done - results[i].t_submit) * 1e3
                    for i in meas])
    sizes = np.array([made[i][0]["n_bits"] for i in meas])
    by_size = {}
    for name, lo, hi in (("below_2^24", 0, 1 << 24), ("2^24_to_2^27", 1 << 24, 1 << 27),
                         ("from_2^27", 1 << 27, 1 << 40)):
        sel = lat[(sizes >= lo) & (sizes < hi)]
        if sel.size:
            by_size[name] = {"jobs": int(sel.size),
                             "p50_ms": round(float(np.percentile(sel, 50)), 3),
                             "p99_ms": round(float(np.percentile(sel, 99)), 3)}
    t0 = min(results[i].t_submit for i in meas)
    t1 = max(results[i].t_done for i in meas)
    bits = sum(made[i][0]["n_bits"] for i in meas)
    # Busy fraction: time with at least one admitted, unfinished job.
    spans = sorted((results[i].t_admit, results[i].t_done) for i in meas)
    busy, cur0, cur1 = 0.0, spans[0][0], spans[0][1]
    for a0, a1 in spans[1:]:
        if a0 > cur1:
            busy += cur1 - cur0
            cur0, cur1 = a0, a1
        else:
            cur1 = max(cur1, a1)
    busy += cur1 - cur0
    queued = np.array([(results[i].t_admit - results[i].t_submit) * 1e3
                       for i in meas])
    offered = bits / (jobs[-1]["arrival_s"] - jobs[args.serve_warmup]["arrival_s"])
    return {"workload": "serving", "jobs": len(meas),
            "warmup_jobs": args.serve_warmup, "rate_hz": cfg["rate_hz"],
            "budget_mib": args.serve_budget_mib,
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3),
            "p99_queue_ms": round(float(np.percentile(queued, 99)), 3),
            "latency_by_size": by_size,
            "sustained_gbps": round(bits / (t1 - t0) / 1e9, 3),
            "offered_gbps": round(offered / 1e9, 3),
            "busy_frac": round(busy / (t1 - t0), 4),
            "ok": sum(1 for i in meas if results[i].status == 0),
            "aborted": sum(1 for i in meas if results[i].status == -2),
            "errors": sum(1 for i in meas if results[i].status not in (0, -2)),
            "oracle_checked_jobs": checked, "oracle_digests_equal": equal}


def serving_digest_check(made, results):
    """Every job of the stream that the oracle's digest file covers (all
    jobs below 2^24 input bits and 20 larger ones) against the oracle's
    SHA-256 of its whole output."""
    ref = load_digests().get("serving")
    if not ref or len(made) != ref["stream_jobs"]:
        return 0, None
    equal = True
    for idx in ref["checked"]:
        want = ref["jobs"].get(str(idx))
        if want is None:
            return 0, None
        r = results[idx]
        if want["status"] == "abort":
            equal = equal and r.status == -2
            continue
        equal = (equal and r.status == 0 and r.out_bits == want["bits"] and
                 words_digest(to_host(made[idx][2]), r.out_bits) == want["sha256"])
    return len(ref["checked"]), equal


# -------------------------------------------------------------- cpu oracle

def spot_check(res, n_rows: int = 24) -> bool:
    """A few output rows of the batched step against the oracle."""
    import oracle
    mlen = res["mlen"]
    osub, oln, owo, _ = res["oracle_sampled"]
    seed = to_host(res["seed"])
    got = to_host(res["out"])
    ooff = np.concatenate([[0], np.cumsum(mlen)[:-1]])
    rng = np.random.default_rng(1)
    for _ in range(n_rows):
        j = int(rng.integers(0, len(mlen)))
        r = int(rng.integers(0, int(mlen[j])))
        want = oracle.toeplitz_rowwin(osub[int(owo[j]):], int(oln[j]), seed,
                                      res["seed_bits"], 0, res["cap"], r)
        k = int(ooff[j]) + r
        if ((int(got[k >> 6]) >> (k & 63)) & 1) != want:
            return False
    return True


def cpu_baseline(res, k_sub: int):
    """The oracle on the host: sampling of the whole input plus the hash of
    k_sub of the sub-blocks, scaled to the full step."""
    import oracle
    c = res["c"]
    n, ns = res["n"], res["ns"]
    log("cpu baseline: oracle sampling of the whole input")
    t0 = time.perf_counter()
    osub, oln, owo, _ = oracle.sample(res["a"], n, ns, oracle.SAMPLE_IID,
                                      key=res["key"])
    t1 = time.perf_counter()
    res["oracle_sampled"] = (osub, oln, owo, None)
    om = oracle.out_lengths(oln, oracle.OUT_RATIO, c["out_a"], c["out_b"])
    seed = to_host(res["seed"])
    k = min(k_sub, ns)
    hi = int(owo[k - 1] + (oln[k - 1] + 63) // 64)
    log(f"cpu baseline: oracle hash of {k} of {ns} sub-blocks")
    t2 = time.perf_counter()
    oracle.hash_batch(osub[:hi], oln[:k], owo[:k], om[:k], seed,
                      res["seed_bits"], 0, res["cap"], level=1)
    t3 = time.perf_counter()
    cores = oracle.threads()
    # The same hash sample on one thread (the sampling is serial anyway).
    k1 = max(1, k // 8)
    hi1 = int(owo[k1 - 1] + (oln[k1 - 1] + 63) // 64)
    log(f"cpu baseline: oracle hash of {k1} sub-blocks on one thread")
    oracle.set_threads(1)
    t4 = time.perf_counter()
    oracle.hash_batch(osub[:hi1], oln[:k1], owo[:k1], om[:k1], seed,
                      res["seed_bits"], 0, res["cap"], level=1)
    t5 = time.perf_counter()
    oracle.set_threads(cores)
    t_full = (t1 - t0) + (t3 - t2) * ns / k
    t_one = (t1 - t0) + (t5 - t4) * ns / k1
    return {
        "value": round(n / t_full / 1e9, 6),
        "unit": "Gbit/s",
        "cores": cores,
        "kind": "oracle",
        "value_1thread": round(n / t_one / 1e9, 6),
        "sample": (f"oracle sampling of all {n} bits ({t1 - t0:.2f} s, one "
                   f"thread) + row-window hash of {k}/{ns} sub-blocks "
                   f"({t3 - t2:.2f} s on {cores} threads; {k1} sub-blocks "
                   f"{t5 - t4:.2f} s on one), hash time scaled to all {ns}"),
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--single-steps", type=int, default=2)
    ap.add_argument("--kernel", default="auto",
                    choices=["auto", "valu", "mfma", "fft"],
                    help="hash kernel of the batched step (auto = tuned)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--fft-chunk", type=int, default=0,
                    help="force the FFT hash's transforms per chunk (0 = tuned)")
    ap.add_argument("--cpu-subblocks", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-single", action="store_true")
    ap.add_argument("--skip-independent", action="store_true")
    ap.add_argument("--skip-contraction", action="store_true")
    ap.add_argument("--skip-small", action="store_true")
    ap.add_argument("--skip-serving", action="store_true")
    ap.add_argument("--skip-table1", action="store_true")
    ap.add_argument("--table1-rows", default=None,
                    help="comma-separated Table I rows (default all five)")
    ap.add_argument("--table1-reps", type=int, default=2)
    ap.add_argument("--serve-jobs", type=int, default=3000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-budget-mib", type=int, default=512)
    ap.add_argument("--mode", default="full",
                    choices=["full", "hash-batched", "hash-independent",
                             "hash-single", "copy", "gather",
                             "contraction", "small", "serving", "table1"],
                    help="full = the benchmark line; the others run one "
                         "part only, for profiler passes")
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the path is not sharded over several GPUs.", file=sys.stderr)
        return 2

    import torch
    from paper_2308_02856_amd import ssbh
    if args.mode == "copy":
        # A plain device copy of known size (calibrates HBM byte counters).
        nb = args.copy_mib << 20
        a = torch.ones(nb // 8, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        # Rate of the same copy (read + write bytes over event time): what a
        # plain streaming kernel reaches on this HBM.
        ms = float(np.mean(time_events(lambda: b.copy_(a), max(3, args.steps))))
        print(json.dumps({"mode": "copy", "bytes_read": nb, "bytes_written": nb,
                          "launches": args.steps, "ms_per_copy": round(ms, 4),
                          "gbps": round(2 * nb / (ms * 1e-3) / 1e9, 1)}),
              flush=True)
        return 0
    if args.mode == "serving":
        print(json.dumps(run_serving(ssbh, args)), flush=True)
        return 0
    ctx = ssbh.Context(0)
    peak = alu_peak_tbitops(ctx.num_cus)
    if args.mode == "table1":
        ctx = ssbh.Context(0)
        print(json.dumps(run_table1(ctx, ssbh, args)), flush=True)
        ctx.close()
        return 0
    if args.mode == "hash-single":
        single = run_single(ctx, ssbh, args)
        print(json.dumps({"mode": args.mode, "ms_valu": single["ms_valu"],
                          "ms_fft": single["ms_fft"],
                          "fft_equals_valu": single["fft_equals_valu"]}),
              flush=True)
        return 0
    if args.mode == "gather":
        print(json.dumps(run_gather(ctx, ssbh, args)), flush=True)
        return 0
    if args.mode == "contraction":
        print(json.dumps(run_contraction(ctx, ssbh, args, peak)), flush=True)
        return 0
    if args.mode == "small":
        print(json.dumps(run_small(ctx, ssbh, args)), flush=True)
        return 0
    res = run_batched(ctx, ssbh, args)
    if args.mode == "hash-independent":
        print(json.dumps(run_batched_independent(ctx, ssbh, args, res)),
              flush=True)
        return 0
    if args.mode == "hash-batched":
        print(json.dumps({"mode": args.mode, "hash_ms": res["hash_ms"],
                          "sample_ms": res["sample_ms"],
                          "schedule": res["schedule"],
                          "kernel_avg_us": {**kernel_avgs(res["sample_kernels"]),
                                            **kernel_avgs(res["hash_kernels"])}}),
              flush=True)
        return 0
    single = None if args.skip_single else run_single(ctx, ssbh, args)
    indep = (None if args.skip_independent else
             run_batched_independent(ctx, ssbh, args, res))

    hk = res["hash_kernels"]
    if res["schedule"].startswith("fft"):
        # The hash's largest pass: the row pass.  Per launch it reads and writes the
        # transforms of its chunk (L complex doubles per transform each way;
        # a transform holds 2 or 4 sub-blocks, "x<k>" in the schedule) and
        # reads the seed spectrum once.
        kern = "k_fft_rows"
        n_l, ms = hk[kern]
        L, per, pb = fft_schedule_parts(res["schedule"])
        transforms = (res["ns"] + per - 1) // per
        per_transform = 2 * L * pb
        total_bytes = (res["timed_calls"] * transforms * per_transform +
                       n_l * L * 16)
        achieved = total_bytes / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": kern, "schedule": res["schedule"],
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": load_traffic(kern, "batched", res["schedule"]),
                "avg_launch_us": round(ms * 1e3 / n_l, 2),
                "algorithmic_bytes_per_launch": int(total_bytes / n_l)}
        dtype = "f64"
    elif res["schedule"].startswith("mfma"):
        kern = "k_toeplitz_mfma"
        n_l, ms = hk[kern]
        achieved = 2 * res["work"] / (ms / n_l * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": kern, "schedule": res["schedule"],
                "achieved": round(achieved, 1), "peak": INT8_PEAK_TOPS,
                "unit": "TOP/s", "frac": round(achieved / INT8_PEAK_TOPS, 4),
                "traffic": load_traffic(kern, "batched", res["schedule"]),
                "avg_launch_us": round(ms * 1e3 / n_l, 2)}
        dtype = "i8"
    else:
        kern = "k_toeplitz_valu"
        n_l, ms = hk[kern]
        achieved = res["work"] / (ms / n_l * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": kern, "schedule": res["schedule"],
                "achieved": round(achieved, 2), "peak": round(peak, 2),
                "unit": "Tbit-op/s", "frac": round(achieved / peak, 4),
                "traffic": load_traffic(kern, "batched", res["schedule"]),
                "avg_launch_us": round(ms * 1e3 / n_l, 2)}
        dtype = "u32"
    copy_gbps = copy_rate_gbps()
    if roof.get("unit") == "GB/s":
        roof["frac_of_plain_copy"] = round(roof["achieved"] / copy_gbps, 4)
    line = {
        "metric": METRIC,
        "value": round(res["n"] / (res["ms_step"] * 1e-3) / 1e9, 4),
        "unit": "Gbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": "batched", "n_bits": res["n"],
                   "n_sub": res["ns"], "p": res["c"]["p"],
                   "sampling": "iid", "out_len": "floor(2*n_j/5)",
                   "seed": "shared", "seed_bits": res["seed_bits"],
                   "bit_products": res["work"],
                   "l_ub": res["l_ub"], "abort_eps": 1e-8,
                   "hash_kernel": res["schedule"]},
        "hash_only_gbps": round(res["n"] / (res["hash_ms"] * 1e-3) / 1e9, 4),
        "hash_ms": round(res["hash_ms"], 4),
        "sample_ms": round(res["sample_ms"], 4),
        "sifted_sample_ms": round(res["sift_ms"], 4),
        "bit_products_per_s": float(f"{res['work'] / (res['hash_ms'] * 1e-3):.4g}"),
        "roofline": roof,
        "plain_copy_gbps": round(copy_gbps, 1),
        "roofline_hash": (fft_hash_roofline(
            res["schedule"], res["ns"], res["n"], int(res["mlen"].sum()),
            res["hash_ms"], True, hk["k_fft_rows"][0] // res["timed_calls"])
            if res["schedule"].startswith("fft") else None),
        "roofline_sampling": sampling_roofline(res),
        "kernel_avg_us": {**kernel_avgs(res["sample_kernels"]),
                          **kernel_avgs(res["hash_kernels"])},
        "tuning": res["tune_report"].strip().splitlines(),
        "oracle_digest_equal": digest_equal("batched", res["out"],
                                            int(res["mlen"].sum())),
    }
    if line["roofline_hash"]:
        line["roofline_hash"]["frac_of_plain_copy"] = round(
            line["roofline_hash"]["achieved"] / copy_gbps, 4)

    if single is not None:
        sg = single["n"] / (single["ms"] * 1e-3) / 1e9
        line["single_block"] = {
            "workload": "single", "n_bits": single["n"], "m_bits": single["m"],
            "gbps": round(sg, 5), "ms": round(single["ms"], 3),
            "ms_valu": round(single["ms_valu"], 3),
            "ms_fft": round(single["ms_fft"], 3),
            "fft_equals_valu": single["fft_equals_valu"],
            "oracle_digest_equal": single["oracle_digest_equal"],
            "valu_alu_frac": round(single["work"] / (single["ms_valu"] * 1e-3)
                                   / 1e12 / peak, 4)}
        line["speedup_vs_single_block"] = round(line["value"] / sg, 2)
    if indep is not None:
        line["batched_independent"] = indep
    if not args.skip_contraction:
        line["contraction"] = run_contraction(ctx, ssbh, args, peak)
    if not args.skip_small:
        line["small"] = run_small(ctx, ssbh, args)
    if not args.skip_table1:
        line["table1"] = run_table1(ctx, ssbh, args)
    ctx.close()
    if not args.skip_serving:
        line["serving"] = run_serving(ssbh, args)
        line["p50_ms"] = line["serving"]["p50_ms"]
        line["p99_ms"] = line["serving"]["p99_ms"]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(res, args.cpu_subblocks)
        line["spot_check_vs_oracle"] = spot_check(res)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
