"""GPU parity at the benchmark's full sizes, in the launch configuration bench.py
times (contiguous work ranges, column aggregation by the th0 rule): the 3D block
matrix (100^3 nodes x 3 dof, 62,460,000 entries) in FP64, FP32 and BF16
storage, its SpMM with k = 8 and 32, the 192^3 Poisson operator and the 4M-row
power-law matrix.  Every row is compared with the oracle where the oracle
finishes in seconds; SpMM and the power-law matrix on seeded samples of rows
(the oracle on the sub-matrix of those rows computes exactly them).  A dyadic
copy of the block matrix must match bit for bit at full size."""
import numpy as np
import pytest

import oracle
from paper_2605_18515_amd import matgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2}


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2605_18515_amd import cbspmv

    torch.cuda.init()
    return cbspmv


@pytest.fixture(scope="module")
def block():
    return matgen.block_3d(100, 3, 10.0, seed=1)


def rows_of(A, rows):
    """The sub-matrix of the given rows (same columns)."""
    rows = np.asarray(rows)
    starts, ends = A.row_ptr[rows], A.row_ptr[rows + 1]
    idx = np.concatenate([np.arange(s, e) for s, e in zip(starts, ends)]) if rows.size else np.zeros(0, np.int64)
    rp = np.concatenate([[0], np.cumsum(ends - starts)]).astype(np.int64)
    return matgen.Csr(rows.size, A.n, rp, A.col_idx[idx], A.values[idx])


def spmv_gpu(cb, A, x, vtype="f64"):
    dt = torch.float64 if vtype == "f64" else torch.float32
    M = cb.CbMatrix.from_csr(A, value_type=vtype)
    xd = torch.from_numpy(x).to("cuda", dt)
    yd = torch.full((A.m,), float("nan"), dtype=dt, device="cuda")
    M.spmv(xd, yd)
    torch.cuda.synchronize()
    info = M.info
    M.close()
    return yd.cpu().double().numpy(), info


def check_rows(y, A, x, vtype, label):
    ref = oracle.spmv(A, x, comp=True)
    scl = oracle.scale(A, x)
    e, viol, worst = oracle.scaled_error(y, ref, scl, TOL[vtype])
    print(f"[{label}] {vtype} rows {A.m} max scaled error {e:.3e}")
    assert viol == 0, f"{label}: {viol} rows above {TOL[vtype]} (max {e}, row {worst})"


@pytest.mark.timeout(300)
@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
def test_block3d_spmv_every_row(cb, block, vtype):
    x = matgen.vector(block.n, 1)
    y, info = spmv_gpu(cb, block, x, vtype)
    assert info["col_agg"] == 1 and info["lb_mode"] == cb.CB_LB_CONTIGUOUS and info["nwaves"] > 1000
    # the quad kernel with 2-byte column offsets from each batch's base
    assert info["spmv_kernel"] == 2 and info["cols16"] == 2
    check_rows(y, block, x, vtype, "block3d 100^3 x 3")


@pytest.mark.timeout(300)
def test_block3d_dyadic_bitwise(cb, block):
    rng = np.random.default_rng(11)
    A = matgen.Csr(block.m, block.n, block.row_ptr, block.col_idx,
                   rng.integers(-64, 65, block.nnz).astype(np.float64) / 64)
    x = rng.integers(-64, 65, block.n).astype(np.float64) / 64
    y, _ = spmv_gpu(cb, A, x, "f64")
    assert np.array_equal(y, oracle.spmv(A, x))


@pytest.mark.timeout(300)
@pytest.mark.parametrize("vtype", ["f32", "bf16"])
@pytest.mark.parametrize("k", [8, 32])
def test_block3d_spmm_sampled_rows(cb, block, k, vtype):
    """The k-right-hand-side product on the FP32 and BF16 copies of the block matrix, X column j
    drawn from seed 3 + j and rounded to FP32, sampled rows against the FP64 oracle on the original
    values and X, within the storage precision's tolerance."""
    X = matgen.rhs_columns(block.n, k, 3)
    M = cb.CbMatrix.from_csr(block, value_type=vtype)
    Xd = torch.from_numpy(X).to("cuda", torch.float32)
    Yd = torch.full((block.m, k), float("nan"), dtype=torch.float32, device="cuda")
    M.spmm(Xd, Yd)
    torch.cuda.synchronize()
    M.close()
    rows = np.sort(np.random.default_rng(7).choice(block.m, 4096, replace=False))
    rows = np.unique(np.concatenate([rows, [0, block.m - 1]]))
    sub = rows_of(block, rows)
    Y = Yd.cpu().double().numpy()[rows]
    ref = oracle.spmm(sub, X)
    scl = oracle.spmm(matgen.Csr(sub.m, sub.n, sub.row_ptr, sub.col_idx, np.abs(sub.values)), np.abs(X))
    e, viol, worst = oracle.scaled_error(Y.ravel(), ref.ravel(), scl.ravel(), TOL[vtype])
    print(f"[block3d spmm {vtype} k={k}] max scaled error {e:.3e} over {rows.size} rows")
    assert viol == 0, (e, worst)


@pytest.fixture(scope="module")
def poisson192():
    return matgen.poisson_3d(192)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
def test_poisson192_every_row(cb, poisson192, vtype):
    """The stencil at scale: FP64 on the streaming kernel, FP32/BF16 on the quad kernel, all reading
    2-byte column offsets from a base per tile (a quad batch spans two grid planes, 73,729 columns)."""
    A = poisson192
    x = matgen.vector(A.n, 1)
    y, info = spmv_gpu(cb, A, x, vtype)
    assert info["col_agg"] == 1 and info["cols16"] == 1
    assert info["spmv_kernel"] == (0 if vtype == "f64" else 2)
    check_rows(y, A, x, vtype, "poisson 192^3")


@pytest.mark.timeout(600)
def test_powerlaw_4m_sampled_rows(cb):
    A = matgen.power_law(4_000_000, seed=2)
    x = matgen.vector(A.n, 1)
    y, _ = spmv_gpu(cb, A, x, "f64")
    # the longest rows (the power law's head) and a seeded sample of the rest
    lens = np.diff(A.row_ptr)
    rows = np.unique(np.concatenate([np.argsort(lens)[-64:],
                                     np.random.default_rng(3).choice(A.m, 20000, replace=False), [0, A.m - 1]]))
    sub = rows_of(A, rows)
    check_rows(y[rows], sub, x, "f64", "power-law 4M (sampled rows)")


def test_powerlaw_literal_sampled_rows(cb):
    """The power-law generator's unscaled row lengths (Zipf 2.1 truncated to [1, 1e5], mean 4.8)."""
    A = matgen.power_law(4_000_000, seed=2, mean_len=None)
    x = matgen.vector(A.n, 1)
    y, _ = spmv_gpu(cb, A, x, "f64")
    lens = np.diff(A.row_ptr)
    rows = np.unique(np.concatenate([np.argsort(lens)[-64:],
                                     np.random.default_rng(4).choice(A.m, 20000, replace=False), [0, A.m - 1]]))
    sub = rows_of(A, rows)
    check_rows(y[rows], sub, x, "f64", "power-law 4M, unscaled lengths (sampled rows)")


@pytest.mark.timeout(300)
@pytest.mark.parametrize("vtype", ["f32", "f64"])
def test_spmm_x_beyond_4gib(cb, vtype):
    """X whose rows lie more than 4 GiB apart in total (a wide leading dimension): the SpMM kernel
    addresses X with 64-bit offsets there and 32-bit ones otherwise; sampled rows against the oracle."""
    A = matgen.block_3d(40, seed=4)
    k, ldx = 8, 6000 if vtype == "f32" else 3000
    dt = torch.float32 if vtype == "f32" else torch.float64
    assert A.n * ldx * (4 if vtype == "f32" else 8) > 2 ** 32
    X = matgen.rhs(A.n, k, 9)
    Xd = torch.zeros((A.n, ldx), dtype=dt, device="cuda")
    Xd[:, :k] = torch.from_numpy(X).to("cuda", dt)
    Yd = torch.full((A.m, k), float("nan"), dtype=dt, device="cuda")
    M = cb.CbMatrix.from_csr(A, value_type=vtype)
    M.spmm(Xd[:, :k], Yd)
    torch.cuda.synchronize()
    M.close()
    del Xd
    rows = np.unique(np.concatenate([np.random.default_rng(8).choice(A.m, 3000, replace=False), [0, A.m - 1]]))
    sub = rows_of(A, rows)
    Xr = X if vtype == "f64" else X.astype(np.float32).astype(np.float64)
    ref = oracle.spmm(sub, Xr)
    scl = oracle.spmm(matgen.Csr(sub.m, sub.n, sub.row_ptr, sub.col_idx, np.abs(sub.values)), np.abs(Xr))
    e, viol, _ = oracle.scaled_error(Yd.cpu().double().numpy()[rows].ravel(), ref.ravel(), scl.ravel(), TOL[vtype])
    print(f"[spmm wide ldx {vtype}] max scaled error {e:.3e}")
    assert viol == 0
