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
