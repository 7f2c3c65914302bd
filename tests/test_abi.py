"""CPU checks of the C ABI: the library loads, exports every declared
function, and host-visible argument errors come back as status codes
(no GPU needed: these calls fail validation before touching a device)."""

import ctypes
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_declares_the_boundary():
    from paper_2308_02856_amd import ssbh
    names = ssbh.header_functions()
    for want in ("ssbh_create", "ssbh_destroy", "ssbh_last_error",
                 "ssbh_sample", "ssbh_hash_batch", "ssbh_seed_from_key",
                 "ssbh_set_schedule"):
        assert want in names, want


def test_library_exports_every_declared_symbol():
    from paper_2308_02856_amd import ssbh
    lib = ctypes.CDLL(ssbh.LIB_PATH)
    missing = [n for n in ssbh.header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_null_context_is_an_error_not_a_crash():
    from paper_2308_02856_amd import ssbh
    L = ssbh.lib()
    rc = L.ssbh_sample(None, None, 0, 1, 0, 0, None, 0, None, 0, None, None,
                       None, None)
    assert rc == ssbh.E_INVAL
    assert b"ctx" in L.ssbh_last_error()
    rc = L.ssbh_hash_batch(None, None, 0, None, None, 0, 0, 0, 1, None, None,
                           0, 0, 0, 0, None, 0, None, None, None)
    assert rc == ssbh.E_INVAL
    L.ssbh_destroy(None)


def test_oracle_is_not_linked_into_the_library():
    from paper_2308_02856_amd import ssbh
    lib = ctypes.CDLL(ssbh.LIB_PATH)
    assert not hasattr(lib, "ssbo_splitmix64")
    src = os.path.join(ROOT, "paper_2308_02856_amd")
    for dirpath, _, files in os.walk(src):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2308_02856_amd import ssbh
    monkeypatch.setattr(ssbh, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ssbh, "_lib", None)
    with pytest.raises(ImportError):
        ssbh.lib()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message
    before touching the device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
