"""The Python binding refuses CSR arrays shorter than what the library reads
(row_ptr[0..n], col_idx[0..row_ptr[n])) before any library call, so that a
bad array length cannot make the library read past a buffer.  CPU only: the
check runs before the device is touched."""
import numpy as np
import pytest

SL = pytest.importorskip("paper_2608_01907_amd.snaplayout")


def _code(fn, *args, **kw):
    with pytest.raises(SL.LayoutError) as ei:
        fn(*args, **kw)
    return ei.value.code, str(ei.value)


@pytest.mark.parametrize("rp_dtype", [np.int32, np.int64])
def test_create_refuses_short_arrays(rp_dtype):
    rp = np.array([0, 2, 4], rp_dtype)  # row_ptr[2] = 4 edges
    code, msg = _code(SL.layout_create_ex, rp, np.array([1, 0, 1], np.int32), 2, 2, 5, 3, 0)
    assert code == SL.LAYOUT_E_INVALID_ARG and "col_idx holds 3" in msg
    code, msg = _code(SL.layout_create_ex, rp, np.zeros(4, np.int32), 3, 2, 5, 3, 0)
    assert code == SL.LAYOUT_E_INVALID_ARG and "n + 1 = 4" in msg
    code, msg = _code(SL.layout_create_ex, np.array([0, 1, -1], rp_dtype), np.zeros(2, np.int32),
                      2, 2, 5, 3, 0)
    assert code == SL.LAYOUT_E_INVALID_ARG and "row_ptr[n] = -1" in msg


def test_other_entry_points_refuse_short_arrays():
    rp, col = np.array([0, 1, 3], np.int32), np.array([1, 0], np.int32)
    assert _code(SL.layout_create, rp, col, 2, 2, 5, 3, 0)[0] == SL.LAYOUT_E_INVALID_ARG
    assert _code(SL.layout_pmds, rp, col, 2)[0] == SL.LAYOUT_E_INVALID_ARG
    graphs = [{"row_ptr": rp, "col_idx": col, "n": 2, "seed": 0}]
    assert _code(SL.layout_batch_create, graphs, 5, 3)[0] == SL.LAYOUT_E_INVALID_ARG
    assert _code(SL.layout_server_submit, None, rp, col, 2, 5, 3, 0)[0] == SL.LAYOUT_E_INVALID_ARG


def test_degree_negatives_refuse_nnz_past_2_32():
    """Degree-weighted negatives build an alias table whose capacity W = nnz
    must stay below 2^32 (thresholds are own * 2^32 / W).  A host CSR with
    row_ptr[n] = 2^32 is refused before any device work; the library only reads
    row_ptr[n] for the check, so a short col array is safe here (the raw C
    entry point is called, bypassing the binding's length check)."""
    import ctypes
    lib = SL.lib()
    o = SL.layout_opts_init()
    o.neg_weights = SL.LAYOUT_NEG_DEGREE
    rp = np.array([0, 1 << 32], np.int64)
    col = np.zeros(1, np.int32)
    h = ctypes.c_void_p()
    rc = lib.layout_create64(rp.ctypes.data, col.ctypes.data, 1, 2, 5, 3, 0, ctypes.byref(o), 0,
                             ctypes.byref(h))
    assert rc == SL.LAYOUT_E_UNSUPPORTED and not h.value
    assert b"nnz < 2^32" in lib.layout_last_error()
