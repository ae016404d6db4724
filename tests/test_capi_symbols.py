"""The C-ABI library loads and exports every entry point include/akra.h declares (no compute calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "akra.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(akra_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("akra_synth2", "akra_adjoint2", "akra_apply_H", "akra_cg_solve", "akra_cg_solve_b", "akra_rhs",
              "akra_plan_create", "akra_plan_destroy", "akra_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2606_06175_amd import akra
    if not os.path.exists(akra.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    L = ctypes.CDLL(akra.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2606_06175_amd import akra
    monkeypatch.setattr(akra, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(akra, "_lib", None)
    try:
        akra.lib()
    except RuntimeError as e:
        assert "not built" in str(e)
    else:
        raise AssertionError("binding did not raise")
