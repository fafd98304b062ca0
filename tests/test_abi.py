"""The C-ABI library loads and exports every entry point include/newmark.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "newmark.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("nm_newmark_init", "nm_newmark_step", "nm_apply_operator", "nm_precond_apply"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2211_08263_amd import newmark
    if not os.path.exists(newmark.LIB_PATH):
        pytest.skip("libnewmark.so not built")
    lib = ctypes.CDLL(newmark.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(newmark.EXPORTED) == set(_declared())


def test_binding_refuses_to_run_without_the_library(monkeypatch, tmp_path):
    from paper_2211_08263_amd import newmark
    monkeypatch.setattr(newmark, "_lib", None)
    monkeypatch.setattr(newmark, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        newmark.load_library()


def test_library_shares_the_hip_runtime_of_torch():
    """One HIP runtime per process: the library binds to the one PyTorch loaded."""
    from paper_2211_08263_amd import newmark as nmb
    nmb.load_library()
    rts = nmb.hip_runtimes_loaded()
    assert len(rts) == 1, rts
