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


def test_binding_structs_match_header_layout(tmp_path):
    """Every struct the binding passes by pointer has the header's size and
    field offsets (a small C program built with gcc against include/sie.h
    prints them)."""
    import shutil
    import subprocess
    from paper_2003_11679_amd import sie
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"sie_c128": sie.c128, "sie_quad_params": sie.QuadParams, "sie_solver_opts": sie.SolverOpts,
               "sie_report": sie.Report, "sie_job_info": sie.JobInfo}
    lines = ['#include <stdio.h>', '#include "sie.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'    printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
