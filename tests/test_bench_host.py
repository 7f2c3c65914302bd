"""Host-side pieces of bench.py and the committed digest file (no GPU):
the whole-output digest the GPU tests and the bench compute equals the one
the oracle-only script stores, the PMC traffic lookup is guarded by the
kernel source, the FFT hash's algorithmic byte count follows its passes, and
the digest file holds every workload."""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _make_digests():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    try:
        import make_digests
    finally:
        sys.path.pop(0)
    return make_digests


def test_digest_definitions_agree():
    md = _make_digests()
    rng = np.random.default_rng(5)
    for bits in (0, 1, 63, 64, 65, 1000, 4096):
        w = rng.integers(0, 2**63, size=(bits + 63) // 64 + 3, dtype=np.uint64)
        assert bench.words_digest(w, bits) == md.digest(w, bits)
    # Words past ceil(bits / 64) do not enter the digest.
    w = np.arange(8, dtype=np.uint64)
    w2 = w.copy()
    w2[5:] = 77
    assert bench.words_digest(w, 300) == bench.words_digest(w2, 300)


def test_traffic_lookup_is_guarded_by_source_and_schedule():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        data = json.load(fh)
    for key, rec in data.items():
        kernel, workload, schedule = key.split(":", 2)
        got = bench.load_traffic(kernel, workload, schedule)
        if rec["source_digest"] == bench.kernel_source_digest(kernel):
            assert got == rec["hbm_bytes_per_launch"]
        else:
            assert got is None
        assert bench.load_traffic(kernel, workload, schedule + ":x") is None


def test_fft_hash_bytes_follow_the_passes():
    L, ns, per, n_bits, out_bits, launches = 4096, 10, 4, 123456, 7890, 3
    sched = f"fft:2:x{per}:L{L}"
    transforms = 3                       # ceil(10 / 4)
    per_transform = 16 * L + 2 * 16 * L + 16 * L     # cols, rows, out
    want_shared = (transforms * per_transform + n_bits // 8 +
                   3 * out_bits // 8 + 3 * 16 * L + launches * 16 * L)
    r = bench.fft_hash_roofline(sched, ns, n_bits, out_bits, 1.0, True, launches)
    assert r["algorithmic_bytes_per_hash"] == want_shared
    assert abs(r["achieved"] - want_shared / 1e-3 / 1e9) < 0.1
    r2 = bench.fft_hash_roofline(f"fft:2:x1:L{L}", ns, n_bits, out_bits, 2.0,
                                 False, 0)
    assert r2["algorithmic_bytes_per_hash"] == (ns * per_transform + n_bits // 8 +
                                                3 * out_bits // 8)
    assert r2["frac"] == round(r2["achieved"] / bench.HBM_PEAK_GBS, 4)


def test_fft_schedule_strings_with_float_storage():
    """Schedule names carry the transform length, the sub-blocks per
    transform and, with complex floats between the passes, ":f32" (8 bytes a
    point): the whole-hash bytes halve the transform traffic then."""
    assert bench.fft_schedule_parts("fft:42:x4:L196608") == (196608, 4, 16)
    assert bench.fft_schedule_parts("fft:0:x1:L196608:f32") == (196608, 1, 8)
    assert bench.fft_schedule_parts("fft:0:x1:L2147483648") == (1 << 31, 1, 16)
    L, ns, n_bits, out_bits = 196608, 6, 1000, 64
    r16 = bench.fft_hash_roofline(f"fft:0:x1:L{L}", ns, n_bits, out_bits, 1.0,
                                  False, 0)
    r8 = bench.fft_hash_roofline(f"fft:0:x1:L{L}:f32", ns, n_bits, out_bits,
                                 1.0, False, 0)
    rest = n_bits // 8 + 3 * out_bits // 8
    assert r16["algorithmic_bytes_per_hash"] == ns * 64 * L + rest
    assert r8["algorithmic_bytes_per_hash"] == ns * 32 * L + rest


def test_digest_file_is_complete():
    with open(os.path.join(HERE, "golden", "digests.json")) as fh:
        d = json.load(fh)
    for part in ("single", "batched", "batched_independent", "contraction"):
        assert len(d[part]["sha256"]) == 64 and d[part]["bits"] > 0, part
    s = d["serving"]
    assert s.get("complete") is True
    assert len(s["checked"]) == len(s["jobs"]) > 1000
    for idx in s["checked"]:
        rec = s["jobs"][str(idx)]
        assert rec["status"] in ("ok", "abort")
        if rec["status"] == "ok":
            assert len(rec["sha256"]) == 64
