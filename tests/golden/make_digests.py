#!/usr/bin/env python3
"""Write the oracle's full-output digests of the benchmark workloads.

Calls only the CPU oracle (oracle/) and the seeded input generators
(workloads/).  For each workload it runs the whole path of the method on the
benchmark's exact inputs -- sampling (Sec. III.B step 1) with the abort rule
(Sec. III.B step 2, Sec. III.D), the per-sub-block Toeplitz hash (Sec. I,
Sec. III.B step 3) and the concatenation (Sec. III.B step 4) -- and stores
the SHA-256 of the whole output (the little-endian bytes of its
ceil(bits / 64) words, tail bits zero) with its length in bits:

* single       one block, 2^24 uniform bits -> 2^23 bits;
* batched      2^28 Bernoulli(0.3) bits, i.i.d. over 2048 sub-blocks,
               floor(2 n_j / 5) bits each, one shared seed;
* batched_independent  the same with an independent seed window per
               sub-block (stride max n_j + max m_j - 1);
* contraction  2^30 uniform bits, keyed permutation, 8192 x 2^17 -> 2^16;
* serving      every job of the benchmark's 3200-job stream with fewer than
               2^24 input bits, plus 20 larger ones drawn with a fixed seed.

The GPU tests hash the library's outputs the same way and compare.  Run:
    python tests/golden/make_digests.py [single batched contraction serving]
(about half an hour on 8 cores; each part is written as soon as it is done).
"""

from __future__ import annotations

import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import (bernoulli_bits, config, serving_input,  # noqa: E402
                       serving_jobs, serving_planes, uniform_bits)

OUT = os.path.join(HERE, "digests.json")
SERVING_JOBS = 3200          # the benchmark's 200 warm-up + 3000 measured jobs
SERVING_SMALL = 1 << 24      # every job below this many input bits is checked
SERVING_LARGE = 20           # and this many larger ones
SERVING_PICK_SEED = 2308


def digest(words: np.ndarray, bits: int) -> str:
    nw = (int(bits) + 63) // 64
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64)[:nw])
    return hashlib.sha256(w.astype("<u8").tobytes()).hexdigest()


def log(msg: str) -> None:
    print(f"[digests] {msg}", flush=True)


def single() -> dict:
    c = config("single")
    n, m = c["n_bits"], c["out_a"]
    x = uniform_bits(n, c["input_seed"])
    seed_bits = n + m - 1
    seed = uniform_bits(seed_bits, c["seed_seed"])
    out = oracle.toeplitz(x, n, seed, seed_bits, m)
    return {"sha256": digest(out, m), "bits": m}


def batched() -> dict:
    c = config("batched")
    n, ns, key = c["n_bits"], c["n_sub"], c["sample_key"]
    a = bernoulli_bits(n, c["p"], c["input_seed"])
    # Abort threshold from the Sec. III.D tail bound, as the benchmark uses.
    l_ub = oracle.ub_threshold(n, 1.0 / ns, ns, 1e-8)
    sub, ln, wo, abort = oracle.sample(a, n, ns, oracle.SAMPLE_IID, key=key,
                                       l_ub=l_ub)
    assert not abort
    om = oracle.out_lengths(ln, oracle.OUT_RATIO, c["out_a"], c["out_b"])
    cap = int(om.max())
    seed_bits = int(ln.max()) + cap - 1
    seed = uniform_bits(seed_bits, c["seed_seed"])
    out, total = oracle.hash_batch(sub, ln, wo, om, seed, seed_bits, 0, cap)
    return {"sha256": digest(out, total), "bits": total, "l_ub": l_ub,
            "seed_bits": seed_bits,
            "sub_sha256": digest(sub, 64 * int(sub.size))}


def batched_independent() -> dict:
    """The batched workload with the paper's independent seeds: sub-block
    j's Toeplitz matrix comes from its own seed window at stride
    S = max n_j + max m_j - 1 (Sec. III.B step 3)."""
    c = config("batched")
    n, ns, key = c["n_bits"], c["n_sub"], c["sample_key"]
    a = bernoulli_bits(n, c["p"], c["input_seed"])
    l_ub = oracle.ub_threshold(n, 1.0 / ns, ns, 1e-8)
    sub, ln, wo, abort = oracle.sample(a, n, ns, oracle.SAMPLE_IID, key=key,
                                       l_ub=l_ub)
    assert not abort
    om = oracle.out_lengths(ln, oracle.OUT_RATIO, c["out_a"], c["out_b"])
    cap = int(om.max())
    stride = int(ln.max()) + cap - 1
    seed_bits = ns * stride
    seed = uniform_bits(seed_bits, c["indep_seed_seed"])
    out, total = oracle.hash_batch(sub, ln, wo, om, seed, seed_bits, stride,
                                   cap)
    return {"sha256": digest(out, total), "bits": total, "stride": stride,
            "seed_bits": seed_bits}


def contraction() -> dict:
    c = config("contraction")
    n, ns, L, m = c["n_bits"], c["n_sub"], c["sub_bits"], c["out_a"]
    a = uniform_bits(n, c["input_seed"])
    perm = oracle.permutation(n, c["perm_key"])
    perm_sha = hashlib.sha256(perm.astype("<u4").tobytes()).hexdigest()
    sub, ln, wo, _ = oracle.sample(a, n, ns, oracle.SAMPLE_PERMUTE,
                                   assign=perm)
    del perm, a
    seed_bits = L + m - 1
    seed = uniform_bits(seed_bits, c["seed_seed"])
    out, total = oracle.hash_batch(sub, ln, wo, np.full(ns, m, np.uint64),
                                   seed, seed_bits, 0, m)
    return {"sha256": digest(out, total), "bits": total,
            "perm_sha256": perm_sha}


def serving_job_sizes(n: int, ns: int, a: int, b: int) -> tuple[int, int, int, int]:
    """The sizes the library derives from a serving job without l_ub (the
    rule stated with ssbh_submit): l_ub = ceil(n/N_S + 8 sqrt(n/N_S)) + 64,
    n_cap = min(l_ub, n), m_cap = floor(n_cap a / b), seed stride
    S = n_cap + m_cap - 1 and N_S S seed bits."""
    mean = n / ns
    l_ub = math.ceil(mean + 8.0 * math.sqrt(mean)) + 64
    n_cap = min(l_ub, n)
    m_cap = (n_cap * a) // b
    stride = n_cap + (m_cap - 1 if m_cap else 0)
    return l_ub, m_cap, stride, ns * stride


def serving_checked(jobs: list[dict]) -> list[int]:
    small = [j["index"] for j in jobs if j["n_bits"] < SERVING_SMALL]
    large = [j["index"] for j in jobs if j["n_bits"] >= SERVING_SMALL]
    rng = np.random.Generator(np.random.PCG64(SERVING_PICK_SEED))
    pick = sorted(rng.choice(large, size=min(SERVING_LARGE, len(large)),
                             replace=False).tolist())
    return sorted(small + pick)


def serving(prev: dict | None) -> dict:
    cfg = config("serving")
    jobs = serving_jobs(SERVING_JOBS, seed=cfg["stream_seed"],
                        rate_hz=cfg["rate_hz"], log2_n=cfg["log2_n"],
                        log2_sub=cfg["log2_sub"], q=cfg["q"], p=cfg["p"])
    planes = serving_planes()
    checked = serving_checked(jobs)
    done = dict(prev["jobs"]) if prev else {}
    t0 = time.time()
    for k, idx in enumerate(checked):
        if str(idx) in done:
            continue
        jb = jobs[idx]
        n, ns = jb["n_bits"], jb["n_sub"]
        a, b = jb["ratio_num"], jb["ratio_den"]
        l_ub, m_cap, stride, seed_bits = serving_job_sizes(n, ns, a, b)
        bits = serving_input(jb, planes)
        sub, ln, wo, abort = oracle.sample(bits, n, ns, oracle.SAMPLE_IID,
                                           key=jb["sample_key"], l_ub=l_ub)
        if abort:
            done[str(idx)] = {"status": "abort"}
        else:
            om = oracle.out_lengths(ln, oracle.OUT_RATIO, a, b)
            seed = oracle.seed_from_key(jb["seed_key"], seed_bits)
            out, total = oracle.hash_batch(sub, ln, wo, om, seed, seed_bits,
                                           stride, m_cap)
            done[str(idx)] = {"status": "ok", "bits": total,
                              "sha256": digest(out, total)}
        if k % 100 == 0:
            log(f"serving: {k + 1}/{len(checked)} jobs ({time.time() - t0:.0f} s)")
            yield {"stream_jobs": SERVING_JOBS, "checked": checked, "jobs": done}
    yield {"stream_jobs": SERVING_JOBS, "checked": checked, "jobs": done,
           "complete": True}


def main(parts: list[str]) -> None:
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for part in parts:
        t0 = time.time()
        log(f"{part}: start")
        if part == "serving":
            for snap in serving(data.get("serving")):
                data["serving"] = snap
                json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
        else:
            data[part] = {"single": single, "batched": batched,
                          "batched_independent": batched_independent,
                          "contraction": contraction}[part]()
            json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
        log(f"{part}: done in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main(sys.argv[1:] or ["single", "batched", "batched_independent",
                          "contraction", "serving"])
