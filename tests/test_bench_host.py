"""Host-side pieces of the benchmark (no GPU): the refusal of more than one GPU, the kernel source
hash, and the rule that committed HBM counters are reported only for the kernel source and the
structure they were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)


def test_kernel_hash_ignores_comments():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0


def test_committed_traffic_applies_only_to_its_structure():
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    for key in ("nnz", "spmv_bytes", "bytes_per_launch", "kernel_source_sha256_16", "fetch_kib", "write_kib"):
        assert key in t
    if t["kernel_source_sha256_16"] != bench.kernel_source_hash():
        pytest.skip("the committed counters predate the current kernel source")
    assert bench.measured_traffic(t["nnz"], t["spmv_bytes"]) == t["bytes_per_launch"]
    assert bench.measured_traffic(t["nnz"] + 1, t["spmv_bytes"]) is None
    assert bench.measured_traffic(t["nnz"], t["spmv_bytes"] + 1) is None
    # the bytes follow from the counters and the copy-kernel factors
    b = t["fetch_kib"] * 1024 * t["fetch_factor"] + t["write_kib"] * 1024 * t["write_factor"]
    assert abs(b - t["bytes_per_launch"]) <= 1024


def test_sampled_rows_give_exactly_those_rows_of_the_product():
    """The bench checks SpMM legs on sampled rows: the oracle's product of the row sub-matrix must be
    exactly the sampled rows of the full product (same summation per row)."""
    import numpy as np

    import oracle
    from paper_2605_18515_amd import matgen

    A = matgen.power_law(3000, seed=5, max_len=200)
    rows = bench.sample_rows(A, 300, 1)
    assert rows[0] == 0 and rows[-1] == A.m - 1 and np.all(np.diff(rows) > 0)
    assert np.diff(A.row_ptr)[rows].max() == np.diff(A.row_ptr).max()
    sub = bench.rows_of(A, rows)
    X = matgen.rhs_columns(A.n, 3, 3)
    assert np.array_equal(oracle.spmm(sub, X), oracle.spmm(A, X)[rows])
    # column j of the block is the vector of seed 3 + j
    assert np.array_equal(matgen.rhs_columns(A.n, 5, 3)[:, :3], X)
