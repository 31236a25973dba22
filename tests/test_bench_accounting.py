"""The benchmark's algorithmic-byte count, on a graph small enough to count
by hand (CPU only)."""
import numpy as np

import bench


def test_algorithmic_bytes_hand_count():
    # rows of degree 2, 1, 0, 2; k = 2; rows longer than hub = 1 edge split
    # into one run per edge; 3 chunks
    row_ptr = np.array([0, 2, 3, 3, 5])
    edges = 5 * (4 + 2 * 8 * (1 + 2))   # col entry + (1 + k) read-modify-writes
    runs = (2 + 1 + 0 + 2) * 2 * 8      # source read and commit per run
    table = 3 * (8 + 4)                 # chunk first edge and source row
    rows = 5 * 8                        # 64-bit row pointers, n + 1 of them
    assert bench.algorithmic_bytes(row_ptr, 4, 2, 1, 3) == edges + runs + table + rows == 416


def test_algorithmic_bytes_3d_and_unsplit_rows():
    row_ptr = np.array([0, 3, 6])       # two rows of 3 edges, no split (hub = 4)
    k = 1
    expect = 6 * (4 + 2 * 16 * (1 + k)) + 2 * 2 * 16 + 1 * 12 + 3 * 8
    assert bench.algorithmic_bytes(row_ptr, 2, k, 4, 1, dim=3) == expect
