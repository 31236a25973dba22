"""The C-ABI library loads on a machine without a GPU and exports every
function that include/snaplayout.h declares (no compute call is made)."""
import os

from paper_2608_01907_amd import _lib


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2608_01907_amd import build

        build.build()
    lib = _lib.load()
    declared = _lib.declared_symbols()
    assert "layout_create" in declared and "layout_epoch" in declared
    assert "layout_get_positions" in declared
    missing = [s for s in declared if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2608_01907_amd import snaplayout as SL

    for name in _lib.declared_symbols():
        assert hasattr(SL, name) or name in ("layout_opts_init",), name


def test_missing_library_is_an_error(tmp_path, monkeypatch):
    import pytest

    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_handle", None)
    with pytest.raises(_lib.LibraryMissing):
        _lib.load()
