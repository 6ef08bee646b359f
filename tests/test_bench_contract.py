"""bench.py's contract pieces that need no GPU.

* The HBM traffic figures (FETCH_SIZE / WRITE_SIZE per product launch) carry
  the hash of the product's sources they were taken on; bench.py reports
  them only while the sources match, so a change to the product without new
  counters would turn every `traffic` field null.  This test fails first.
* The algorithmic bytes of one masked product on the 512^2 workload: A's
  column indices and values, A's and N's row pointers, N's column indices,
  X read once and Z written once, 12 nnz(A) + 20 nnz(N) + 8 (n + 1).
* More than one GPU is refused with a message and exit status 2.
"""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_figures_match_the_sources():
    assert bench.traffic_bytes() == bench.TRAFFIC_BYTES
    for w in bench.OTHER_WORKLOADS:
        assert bench.traffic_bytes(w) == bench.TRAFFIC_OTHER[w], w
    # each measured figure is at least the algorithmic bytes it moves
    assert bench.TRAFFIC_BYTES >= 51806092


def test_headline_algorithmic_bytes():
    n, nnz_a, nnz_n, nc = 262144, 2353156, 1073553, 29241
    b, aux = bench.product_bytes(nnz_a, n, nnz_n, n, n_f=n - nc)
    assert b == 12 * nnz_a + 20 * nnz_n + 8 * (n + 1) == 51806092
    # root flags (1 byte per row), the Bc rows of the roots and the F rows'
    # G^+ (n_B = 1): 9 bytes per row whatever the number of roots
    assert aux == n + 8 * nc + 8 * (n - nc) == 2359296
    # a batch reads the shared structure once and the values, X and Z per problem
    b4, _ = bench.product_bytes(nnz_a, n, nnz_n, n, n_f=n - nc, batch=4)
    assert b4 == b + 3 * (8 * nnz_a + 16 * nnz_n)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
