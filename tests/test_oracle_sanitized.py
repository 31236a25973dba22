"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle is built with -fsanitize=address,undefined into a temporary
directory and driven through its Python wrapper in a child process (the
sanitizer runtime must be preloaded into the interpreter).  Every entry point
runs on small graphs, including the edge cases (an edgeless graph, a two-node
graph, k = 0, a hub, caller weights with zeros, 3D positions); any invalid
access or undefined operation aborts the child with a report.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    import numpy as np
    import synthgraph as S
    from oracle import oracle as O

    O.LIB = {lib!r}
    O._lib = None
    g = S.small_sbm(300, 3, 8.0, 2)
    rp, col, n = g.row_ptr, g.col, g.n
    Y = O.serial_run(rp, col, n, 5, 4, 1)
    Y3 = O.serial_run(rp, col, n, 3, 2, 1, dim=3)
    O.jacobi_epoch(rp, col, n, 5, 1, 4, 1, Y, want_abs=True)
    O.jacobi_epoch(rp, col, n, 4, 0, 4, 1, Y3)
    w = np.random.default_rng(0).integers(0, 9, n)
    w[0] += 1
    thr, alias = O.alias_build(w)
    O.draw_negatives(rp, col, n, 8, 3, 2, mode=O.NEG_DEGREE, thr=thr, alias=alias)
    O.draw_edges(rp, n, 5, 2, 7, np.arange(0, col.size, 11))
    O.sampled_energy(rp, col, n, 5, 1, 1, Y, parts=True)
    O.effective_energy(rp, col, n, 5, Y, parts=True)
    O.threaded_run(rp, col, n, 5, 3, 1, 4)
    O.init_positions_at(n, 3, np.array([0, n - 1]))
    # edge cases: no edges, two nodes, k = 0
    e_rp = np.zeros(6, np.int32)
    O.serial_run(e_rp, np.zeros(0, np.int32), 5, 5, 2, 0)
    O.jacobi_epoch(e_rp, np.zeros(0, np.int32), 5, 5, 0, 2, 0, O.init_positions(5, 0))
    p_rp, p_col = S.csr_from_pairs(np.array([0]), np.array([1]), 2)
    O.serial_run(p_rp, p_col, 2, 3, 5, 4)
    O.draw_negatives(p_rp, p_col, 2, 8, 0, 1)
    O.serial_run(rp, col, n, 0, 2, 1)
    print("sanitized oracle: ok")
""")


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not asan or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call([
        "gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
        "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
        "-fno-omit-frame-pointer", "-o", lib, os.path.join(ROOT, "oracle", "snap_oracle.c"),
        "-lm", "-lpthread"])
    env = dict(os.environ, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    proc = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)], env=env,
                          capture_output=True, text=True, timeout=600)
    assert proc.returncode == 0, proc.stderr[-4000:]
    assert "sanitized oracle: ok" in proc.stdout
