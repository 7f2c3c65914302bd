"""Mutation checks: the oracle's pins reject plausible mistakes.

Each case builds a copy of the oracle (oracle/__init__.py and oracle.c) with
one planted mistake, on the CPU, in a temporary folder, and requires that at
least one of the pins run on the real oracle in tests/test_oracle_pins.py
fails on the copy.  The real oracle is never modified.
"""

from __future__ import annotations

import importlib.util
import inspect
import os
import shutil
import subprocess

import pytest

import oracle
from tests import pin_checks
from tests import test_oracle_pins as pins

ORACLE_DIR = os.path.dirname(os.path.abspath(oracle.__file__))


def mutated_oracle(tmp_path, c_old=None, c_new=None, py_old=None, py_new=None):
    """A fresh copy of the oracle package with one textual change planted in
    oracle.c or oracle/__init__.py, built with gcc into tmp_path."""
    src_c = open(os.path.join(ORACLE_DIR, "oracle.c")).read()
    src_py = open(os.path.join(ORACLE_DIR, "__init__.py")).read()
    if c_old is not None:
        assert src_c.count(c_old) == 1, c_old
        src_c = src_c.replace(c_old, c_new)
    if py_old is not None:
        assert src_py.count(py_old) == 1, py_old
        src_py = src_py.replace(py_old, py_new)
    d = tmp_path / "mut_oracle"
    d.mkdir()
    (d / "oracle.c").write_text(src_c)
    (d / "__init__.py").write_text(src_py)
    lib = str(d / "_oracle.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                           "-std=c11", str(d / "oracle.c"), "-o", lib])
    spec = importlib.util.spec_from_file_location(
        f"mut_oracle_{abs(hash(str(d)))}", str(d / "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._load()
    return mod


def fails(fn, *args) -> bool:
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


# ------------------------------------------------------------- GEAT ---

GEAT_MUTATIONS = {
    "V^2 term doubled": (
        "/ (2.0 * (2.0 - a)) * V * V", "/ (2.0 * (2.0 - a)) * V * V * 2.0"),
    "(alpha-1)/(2-alpha) not squared on K'": (
        "((a - 1.0) / (2.0 - a)) ** 2 * kprime",
        "((a - 1.0) / (2.0 - a)) * kprime"),
    "d_X not squared in V": (
        "math.log2(2.0 * dx * dx + 1.0)", "math.log2(2.0 * dx + 1.0)"),
    "alpha dropped from alpha log2(1/p_Omega)": (
        "a * math.log2(1.0 / p[\"p_omega\"])", "math.log2(1.0 / p[\"p_omega\"])"),
    "ln 2 dropped from the V^2 term": (
        "(a - 1.0) * math.log(2.0) / (2.0 * (2.0 - a))",
        "(a - 1.0) / (2.0 * (2.0 - a))"),
    "cube dropped from ln^3 in K'": (
        "math.log(2.0 ** D + math.e ** 2) ** 3)",
        "math.log(2.0 ** D + math.e ** 2))"),
}


@pytest.mark.parametrize("name", list(GEAT_MUTATIONS))
def test_geat_pins_reject_planted_mistake(name):
    old, new = GEAT_MUTATIONS[name]
    src = inspect.getsource(oracle.geat_key_length)
    assert src.count(old) == 1, name
    ns = dict(oracle.__dict__)
    exec(src.replace(old, new), ns)
    bad = ns["geat_key_length"]
    # The unmodified function passes both checks ...
    pin_checks.check_geat_eq1(oracle.geat_key_length)
    pin_checks.check_geat_expansion(oracle.geat_key_length)
    # ... and the planted mistake fails at least one.
    assert (fails(pin_checks.check_geat_eq1, bad)
            or fails(pin_checks.check_geat_expansion, bad)), name


# ------------------------------------------------------------- V map ---

V_MAP_LINE = "return (uint32_t)(((uint64_t)u * (uint64_t)n_sub) >> 32);"


@pytest.mark.parametrize("name,new", [
    ("u mod N_S", "return u % n_sub;"),
    ("high bits of the wrong half", "u = (uint32_t)(r >> 32); "
     "return (uint32_t)(((uint64_t)u * (uint64_t)n_sub) >> 32);"),
])
def test_v_map_pins_reject_planted_mistake(tmp_path, name, new):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    mod = mutated_oracle(tmp_path, c_old=V_MAP_LINE, c_new=new)
    assert any(fails(pins.test_draw_v_is_a_monotone_even_range_map, mod, ns)
               for ns in (7, 1000))


# ------------------------------------------------------- permutation ---

@pytest.mark.parametrize("name,old,new", [
    ("Sattolo's variant (j < i)",
     "return (uint64_t)(((unsigned __int128)r * (i + 1)) >> 64);",
     "return (uint64_t)(((unsigned __int128)r * i) >> 64);"),
    ("stream index ascending with i",
     "uint64_t r = ssbo_splitmix64(key, n - 1 - i);",
     "uint64_t r = ssbo_splitmix64(key, i);"),
    ("assignment instead of exchange",
     "        perm[j] = t;\n", "\n"),
    ("low word of the product",
     "return (uint64_t)(((unsigned __int128)r * (i + 1)) >> 64);",
     "return (uint64_t)(((unsigned __int128)r * (i + 1)) % (i + 1));"),
])
def test_permutation_pins_reject_planted_mistake(tmp_path, name, old, new):
    mod = mutated_oracle(tmp_path, c_old=old, c_new=new)
    checks = [
        lambda: pins.test_keyed_permutation_is_a_permutation(mod, 1000),
        lambda: pins.test_keyed_permutation_choices(mod),
        lambda: pins.test_keyed_permutation_is_uniform_over_all_orderings(
            mod, 4, 6000),
    ]
    assert any(fails(c) for c in checks), name


# ------------------------------------- Toeplitz, sampling, concatenation ---

def fails_any(fn) -> bool:
    """True when a pin rejects the copy: a failed assertion, or an error
    the copy's wrong arithmetic provokes (a refused argument, say)."""
    try:
        fn()
    except Exception:
        return True
    return False


def toeplitz_pins(mod):
    return [
        lambda: pins.test_toeplitz_exhaustive_tiny_against_clmul(mod),
        lambda: pins.test_toeplitz_against_fft_and_clmul(mod, 100, 37),
        lambda: pins.test_toeplitz_closed_forms(mod),
        lambda: pins.test_toeplitz_ignores_input_bits_past_n(mod),
        lambda: pins.test_row_functions_agree_with_block(mod),
    ]


def sampling_pins(mod):
    return [
        lambda: pins.test_partition_equals_boolean_selection(mod, 10007, 13),
        lambda: pins.test_partition_equals_boolean_selection(mod, 5000, 2048),
        lambda: pins.test_sample_iid_is_partition_by_splitmix_assignment(mod),
    ]


def sifting_pins(mod):
    return [lambda: pins.test_sift_equals_selection_by_v_and_keep(
        mod, 5000, 7, 0.6)]


def batch_pins(mod):
    return [lambda: pins.test_hash_batch_concatenates_per_block_hashes(mod, s)
            for s in ("shared", "independent")]


# (name, text in oracle.c, planted replacement, pins that must catch it).
# Every planted mistake keeps each access inside its buffer, so a copy can
# only give wrong answers, never touch memory it does not own.
C_MUTATIONS = [
    ("Toeplitz: first column dropped",
     "    for (uint64_t c = 0; c < n; ++c)\n        acc ^= get_bit",
     "    for (uint64_t c = 1; c < n; ++c)\n        acc ^= get_bit",
     toeplitz_pins),
    ("Toeplitz: AND of seed and input bit replaced by OR",
     "acc ^= get_bit(seed, base + c - r + cap - 1) & get_bit(x, c);",
     "acc ^= get_bit(seed, base + c - r + cap - 1) | get_bit(x, c);",
     toeplitz_pins),
    ("Toeplitz: XOR accumulation replaced by OR",
     "acc ^= get_bit(seed, base + c - r + cap - 1) & get_bit(x, c);",
     "acc |= get_bit(seed, base + c - r + cap - 1) & get_bit(x, c);",
     toeplitz_pins),
    ("row windows: tail mask of the last input word dropped",
     "if (w == nw - 1 && (n & 63)) xw &= (1ull << (n & 63)) - 1ull;",
     "(void)0;",
     toeplitz_pins),
    ("row windows: window start one bit late",
     "uint64_t start = base + cap - 1 - r, nw",
     "uint64_t start = base + cap - r, nw",
     toeplitz_pins),
    ("row windows: seed window read with the wrong shift",
     "return (lo >> sh) | (hi << (64 - sh));",
     "return (lo << sh) | (hi >> (64 - sh));",
     toeplitz_pins),
    ("sampling: a sub-block's bits in descending order",
     "put_bit(sub, 64ull * word_off[j] + cursor[j], get_bit(a, i));",
     "put_bit(sub, 64ull * word_off[j] + (len[j] - 1 - cursor[j]), get_bit(a, i));",
     sampling_pins),
    ("sampling: word offsets rounded down",
     "        word_off[j] = acc;\n        acc += (len[j] + 63) / 64;",
     "        word_off[j] = acc;\n        acc += len[j] / 64;",
     sampling_pins),
    ("sifting: the flag stored instead of the data bit",
     "put_bit(out, 64ull * out_off[j] + pos, get_bit(sub, b));",
     "put_bit(out, 64ull * out_off[j] + pos, get_bit(keep_sub, b));",
     sifting_pins),
    ("concatenation: output offset never advanced",
     "        if (rc) return -1;\n        off += out_len[j];",
     "        if (rc) return -1;",
     batch_pins),
    ("concatenation: the seed offset of sub-block j + 1",
     "uint64_t base = (uint64_t)j * stride;",
     "uint64_t base = (uint64_t)(j + 1 < n_sub ? j + 1 : j) * stride;",
     batch_pins),
    ("output lengths rounded up",
     "out_len[j] = (uint64_t)(p / b);",
     "out_len[j] = (uint64_t)((p + b - 1) / b);",
     lambda mod: [lambda: pins.test_out_lengths(mod)]),
    ("seed tail not masked",
     "    if (n_bits & 63) seed[nw - 1] &= (1ull << (n_bits & 63)) - 1ull;\n}",
     "}",
     lambda mod: [lambda: pins.test_seed_from_key(mod)]),
]


@pytest.mark.parametrize("name,old,new,checks", C_MUTATIONS,
                         ids=[c[0] for c in C_MUTATIONS])
def test_core_pins_reject_planted_mistake(tmp_path, name, old, new, checks):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    # The real oracle passes the same pins ...
    assert not any(fails_any(c) for c in checks(oracle)), name
    # ... and the copy with the planted mistake fails at least one.
    mod = mutated_oracle(tmp_path, c_old=old, c_new=new)
    assert any(fails_any(c) for c in checks(mod)), name
