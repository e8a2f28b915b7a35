"""C-ABI boundary checks that need no GPU: the library loads and exports every function
that include/taccel.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "taccel.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(taccel_[a-z_]+)\s*\(", src)))


def test_header_declares_boundary():
    names = _declared()
    for required in ("taccel_scene_create", "taccel_step", "taccel_state_read",
                     "taccel_state_write", "taccel_scene_destroy", "taccel_batch_create",
                     "taccel_batch_step", "taccel_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2504_12908_amd import taccel
    if not os.path.exists(taccel.LIB_PATH):
        pytest.skip("libtaccel.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(taccel.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.taccel_status_str.restype = ctypes.c_char_p
    assert lib.taccel_status_str(0) == b"OK"
    assert lib.taccel_status_str(4) == b"LINESEARCH_FAILED"


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    from paper_2504_12908_amd import taccel
    monkeypatch.setattr(taccel, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(taccel, "_lib", None)
    with pytest.raises(RuntimeError):
        taccel.lib()
