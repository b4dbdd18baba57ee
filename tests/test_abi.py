"""CPU checks of the C ABI: the library loads, exports every entry point that
include/sie.h declares, and the binding's signature table covers them."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sie.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sie_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    assert "sie_matvec" in names and "sie_solve" in names and len(names) >= 25


def test_library_exports_every_declared_symbol():
    from paper_2003_11679_amd.sie import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.fail("libsie.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2003_11679_amd.sie import SIGNATURES
    bound = {s[0] for s in SIGNATURES}
    assert set(declared()) == bound


def test_no_device_is_a_clean_error():
    """Without a HIP device the context call fails with SIE_EDEVICE (no fault)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_2003_11679_amd import Context, SieError
    with pytest.raises(SieError) as e:
        Context(0)
    assert e.value.status == -6


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import paper_2003_11679_amd.sie as S
    monkeypatch.setattr(S, "_lib", None)
    monkeypatch.setattr(S, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError):
        S.lib()
