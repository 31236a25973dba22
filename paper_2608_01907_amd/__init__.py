"""SNAP-tFDP edge-centric layout on MI355X (gfx950).

The layout runs in libsnaplayout.so (hand-written HIP kernels behind a C ABI,
include/snaplayout.h); this package only binds it."""
from . import snaplayout  # noqa: F401
from .snaplayout import Layout, LayoutError  # noqa: F401
