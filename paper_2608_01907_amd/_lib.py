"""Loader of the in-tree HIP library.  There is no fallback: when the shared
library is missing the import of any entry point raises."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsnaplayout.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "snaplayout.h")

_handle = None
_configured = set()


class LibraryMissing(ImportError):
    pass


def load(signatures: dict | None = None):
    """Loads libsnaplayout.so once and applies ctypes signatures."""
    global _handle
    if _handle is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} is not built; run paper_2608_01907_amd/build.py "
                "(or __graft_entry__.build()) first")
        # PyTorch ships its own HIP runtime.  Loading torch first makes this
        # library bind to that same runtime, so that one process never holds
        # two (torch then finds no device when it starts after this library).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        _handle = ctypes.CDLL(LIB_PATH)
    if signatures:
        for name, (res, args) in signatures.items():
            if name in _configured:
                continue
            fn = getattr(_handle, name)
            fn.restype = res
            fn.argtypes = args
            _configured.add(name)
    return _handle


def declared_symbols(header: str = HEADER) -> list[str]:
    """Function names declared in a public header (for the export check)."""
    import re

    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)
    keywords = {"if", "sizeof", "return", "defined"}
    out = []
    for nm in names:
        if nm in keywords or nm in out:
            continue
        out.append(nm)
    return out
