"""GPU parity of 8 x 8 tiles (tile_dim = 8), the library's second sub-block size: every kernel that
takes a natural-order or Algorithm 2 structure (the streaming kernel, the quad kernel, the
tile-at-a-time kernel, both k-right-hand-side kernels, the serving loop's batched launch) against
the CPU oracle, to the tolerances of the 16 x 16 tests: FP64 1e-12, FP32 1e-5, BF16 1e-2 of
|alpha||A||x| + |beta||y0|, and bit for bit on exact-arithmetic inputs."""
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


MATS = {
    "lap64": lambda: matgen.laplacian_2d(64),
    "lap13": lambda: matgen.laplacian_2d(13),
    "block8": lambda: matgen.block_3d(8, seed=1),
    "poisson12": lambda: matgen.poisson_3d(12),
    "power": lambda: matgen.power_law(20000, seed=2, max_len=5000, window=500),
    "rect": lambda: matgen.random_csr(300, 517, 0.05, 4),
    "wide": lambda: matgen.random_csr(37, 4000, 0.3, 5),
    "dense_mix": lambda: matgen.from_dense(
        np.where(np.random.default_rng(1).random((170, 190)) < np.repeat([0.95, 0.4, 0.05], [64, 60, 46])[:, None],
                 np.random.default_rng(2).uniform(-1, 1, (170, 190)), 0.0)),
}


def run_spmv(cb, A, x, alpha=1.0, beta=0.0, y0=None, vtype="f64", **opts):
    dt = torch.float64 if vtype == "f64" or opts.get("vector_f64") else torch.float32
    M = cb.CbMatrix.from_csr(A, value_type=vtype, tile_dim=8, **opts)
    assert M.info["tile_dim"] == 8
    xd = torch.from_numpy(np.asarray(x, dtype=np.float64)).to("cuda", dt)
    if y0 is None:
        yd = torch.full((A.m,), float("nan"), dtype=dt, device="cuda")
    else:
        yd = torch.from_numpy(np.asarray(y0, dtype=np.float64)).to("cuda", dt)
    M.spmv(xd, yd, alpha, beta)
    torch.cuda.synchronize()
    out = yd.cpu().double().numpy()
    M.close()
    return out


def check(cb, A, x, alpha=1.0, beta=0.0, y0=None, vtype="f64", label="", **opts):
    y = run_spmv(cb, A, x, alpha, beta, y0, vtype, **opts)
    ref = oracle.spmv(A, x, alpha, beta, y0, comp=True)
    e, viol, worst = oracle.scaled_error(y, ref, oracle.scale(A, x, alpha, beta, y0), TOL[vtype])
    print(f"[8x8 {label}] {vtype} {opts} max scaled error {e:.3e}")
    assert viol == 0, f"{label}: {viol} rows above {TOL[vtype]} (max {e}, row {worst}: {y[worst]} vs {ref[worst]})"
    return y


@pytest.mark.parametrize("kernel", [0, 2])
@pytest.mark.parametrize("name", sorted(MATS))
def test_spmv_f64(cb, name, kernel):
    A = MATS[name]()
    x = matgen.vector(A.n, 7)
    y0 = matgen.vector(A.m, 3, stream=matgen.STREAM_Y0)
    for lb in ("contiguous", "none") + (("paper",) if kernel == 0 else ()):
        for agg in (-1, 0, 1):
            check(cb, A, x, label=f"{name} k{kernel} {lb}", lb_mode=lb, col_agg=agg, spmv_kernel=kernel)
        # short work ranges: panels shared between ranges, alpha and beta
        check(cb, A, x, 1.5, -0.5, y0, label=f"{name} k{kernel} {lb} short", lb_mode=lb, wave_nnz=64,
              spmv_kernel=kernel)


@pytest.mark.parametrize("kernel", [0, 2])
@pytest.mark.parametrize("name", ["dense_mix", "power", "block8"])
def test_spmv_formats(cb, name, kernel):
    """th2 = 40 and th2 = 10 give Dense 8 x 8 tiles; th1 = th2 = 1 makes every tile Dense or CSR."""
    A = MATS[name]()
    x = matgen.vector(A.n, 8)
    for th in ((32, 128), (8, 40), (2, 10), (1, 1), (300, 300)):
        for agg in (0, 1):
            for lb in ("contiguous", "paper") if kernel == 0 else ("contiguous",):
                check(cb, A, x, label=f"{name} th={th}", col_agg=agg, th1=th[0], th2=th[1], lb_mode=lb,
                      spmv_kernel=kernel)


@pytest.mark.parametrize("vtype", ["f32", "bf16"])
@pytest.mark.parametrize("rr", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("name", ["block8", "power", "lap64", "dense_mix", "rect"])
def test_low_precision_row_reduce(cb, name, rr, vtype):
    A = MATS[name]()
    x = matgen.vector(A.n, 12)
    y0 = matgen.vector(A.m, 3, stream=matgen.STREAM_Y0)
    for kernel in (0, 2):
        if kernel == 2 and rr == 1:
            continue
        for agg in (0, 1):
            check(cb, A, x, vtype=vtype, label=f"{name} rr={rr} k{kernel}", col_agg=agg, row_reduce=rr, th1=8,
                  th2=40, spmv_kernel=kernel)
        check(cb, A, x, 1.5, -0.5, y0, vtype, label=f"{name} rr={rr} k{kernel} shared", row_reduce=rr,
              wave_nnz=64, spmv_kernel=kernel)
    check(cb, A, x, vtype=vtype, label=f"{name} paper order", lb_mode="paper", th1=8, th2=40)


@pytest.mark.parametrize("vtype", ["f32", "bf16"])
def test_wide_vectors(cb, vtype):
    """FP32/BF16 storage with double x and y: the FP64 oracle on the rounded values to 1e-12."""
    for name in ("block8", "dense_mix", "power"):
        A = MATS[name]()
        vals = oracle.f32_values(A.values) if vtype == "f32" else oracle.bf16_values(A.values)
        Ar = matgen.Csr(A.m, A.n, A.row_ptr, A.col_idx, vals)
        x = matgen.vector(A.n, 13)
        for kernel, lb in ((0, "contiguous"), (2, "contiguous"), (0, "paper")):
            y = run_spmv(cb, A, x, vtype=vtype, vector_f64=1, lb_mode=lb, spmv_kernel=kernel, th1=8, th2=40)
            e, viol, _ = oracle.scaled_error(y, oracle.spmv(Ar, x, comp=True), oracle.scale(Ar, x), 1e-12)
            assert viol == 0, (name, kernel, lb, e)


def test_exact_arithmetic_bitwise(cb):
    """Dyadic values and x: every partial sum exact, so any summation order gives the oracle's bits."""
    for name, A in [("dyadic", matgen.random_csr(500, 700, 0.04, 3, values="dyadic")),
                    ("lap", matgen.laplacian_2d(40)), ("poisson", matgen.poisson_3d(10))]:
        x = matgen.vector(A.n, 4, dyadic=True)
        ref = oracle.spmv(A, x)
        for kernel, lb in ((0, "contiguous"), (0, "none"), (0, "paper"), (2, "contiguous")):
            for agg in (0, 1):
                for th in ((32, 128), (4, 20)):
                    y = run_spmv(cb, A, x, lb_mode=lb, col_agg=agg, th1=th[0], th2=th[1], wave_nnz=64,
                                 spmv_kernel=kernel)
                    assert np.array_equal(y.view(np.uint64), ref.view(np.uint64)), (name, kernel, lb, agg, th)


def test_identity_permutation_and_degenerate(cb):
    x = matgen.vector(1000, 3)
    I = matgen.identity(1000)
    P, pi = matgen.permutation(1000, 3)
    for kernel in (0, 2):
        assert np.array_equal(run_spmv(cb, I, x, spmv_kernel=kernel).view(np.uint64), x.view(np.uint64))
        for agg in (0, 1):
            assert np.array_equal(run_spmv(cb, P, x, col_agg=agg, spmv_kernel=kernel).view(np.uint64),
                                  x[pi].view(np.uint64))
    y0 = np.arange(40, dtype=np.float64)
    E = matgen.Csr(40, 30, np.zeros(41, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert np.array_equal(run_spmv(cb, E, np.ones(30), 1.0, 0.5, y0), 0.5 * y0)
    D = np.zeros((100, 60)); D[3, 5] = 1.0; D[70, 59] = 2.0; D[99, 0] = 3.0
    for lb in ("contiguous", "paper"):
        check(cb, matgen.from_dense(D), matgen.vector(60, 1), 1.0, 2.0, np.ones(100), label="empty panels",
              lb_mode=lb)


def test_nonfinite_x_and_values(cb):
    """Dense 8 x 8 tiles must not multiply their zero fill with an Inf of x."""
    rng = np.random.default_rng(5)
    A = MATS["dense_mix"]()
    vals = A.values.copy()
    vals[rng.integers(0, A.nnz, 20)] = np.nan
    vals[rng.integers(0, A.nnz, 20)] = np.inf
    B = matgen.Csr(A.m, A.n, A.row_ptr, A.col_idx, vals)
    x = matgen.vector(A.n, 5)
    x[rng.integers(0, A.n, 5)] = np.inf
    for th in ((32, 128), (4, 16)):
        for kernel, lb in ((0, "contiguous"), (2, "contiguous"), (0, "paper")):
            for agg in (0, 1):
                check(cb, B, x, label="nonfinite", col_agg=agg, th1=th[0], th2=th[1], lb_mode=lb, spmv_kernel=kernel)


def run_spmm(cb, A, X, alpha, beta, Y0, vtype="f64", ld_pad=0, **opts):
    dt = torch.float64 if vtype == "f64" or opts.get("vector_f64") else torch.float32
    k = X.shape[1]
    M = cb.CbMatrix.from_csr(A, value_type=vtype, tile_dim=8, **opts)
    Xd = torch.zeros((A.n, k + ld_pad), dtype=dt, device="cuda")
    Xd[:, :k] = torch.from_numpy(X).to("cuda", dt)
    Yd = torch.full((A.m, k + ld_pad), 7.0, dtype=dt, device="cuda")
    Yd[:, :k] = torch.from_numpy(Y0).to("cuda", dt)
    M.spmm(Xd[:, :k], Yd[:, :k], alpha, beta)
    torch.cuda.synchronize()
    out = Yd.cpu().double().numpy()
    M.close()
    if ld_pad:
        assert np.all(out[:, k:] == 7.0), "wrote outside the k columns"
    return out[:, :k]


@pytest.mark.parametrize("k", [1, 3, 8, 17, 32, 40])
@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
def test_spmm(cb, k, vtype):
    A = MATS["dense_mix"]() if k % 2 else MATS["block8"]()
    X = matgen.rhs(A.n, k, k)
    Y0 = matgen.rhs(A.m, k, k + 50)
    ref = oracle.spmm(A, X, 1.5, -0.5, Y0, comp=True)
    scl = oracle.spmm_scale(A, X, 1.5, -0.5, Y0)
    for lb, agg, th, wn in (("contiguous", -1, (32, 128), 0), ("paper", 0, (8, 40), 0), ("paper", 1, (2, 10), 0),
                            ("contiguous", 1, (8, 40), 0), ("contiguous", 0, (2, 10), 64), ("none", 1, (8, 40), 64)):
        Y = run_spmm(cb, A, X, 1.5, -0.5, Y0, vtype, ld_pad=3, lb_mode=lb, col_agg=agg, th1=th[0], th2=th[1],
                     wave_nnz=wn)
        e, viol, _ = oracle.scaled_error(Y, ref, scl, TOL[vtype])
        print(f"8x8 spmm k={k} {vtype} {lb} agg={agg} th={th} max scaled error {e:.3e}")
        assert viol == 0, (k, vtype, lb, agg, th, e)


def test_spmm_exact_bitwise(cb):
    A = matgen.random_csr(300, 280, 0.06, 11, values="dyadic")
    X = np.random.default_rng(1).integers(-64, 65, (280, 8)).astype(np.float64) / 64
    ref = oracle.spmm(A, X)
    for th in ((32, 128), (2, 10)):
        for lb in ("contiguous", "paper"):
            Y = run_spmm(cb, A, X, 1.0, 0.0, np.zeros((300, 8)), col_agg=0, th1=th[0], th2=th[1], lb_mode=lb)
            assert np.array_equal(Y.view(np.uint64), ref.view(np.uint64)), (th, lb)


@pytest.mark.parametrize("vtype", ["f64", "f32"])
def test_spmm_dense_tiles_with_nonfinite_x(cb, vtype):
    A = MATS["dense_mix"]()
    k = 16
    X = matgen.rhs(A.n, k, 3)
    X[5, 3] = np.inf
    X[40, 0] = -np.inf
    X[77, 9] = np.nan
    ref = oracle.spmm(A, X, comp=True)
    for th in ((8, 40), (2, 10)):
        for lb in ("contiguous", "paper"):
            Y = run_spmm(cb, A, X, 1.0, 0.0, np.zeros((A.m, k)), vtype, col_agg=0, th1=th[0], th2=th[1], lb_mode=lb)
            e, viol, w = oracle.scaled_error(Y, ref, oracle.spmm_scale(A, X), TOL[vtype])
            assert viol == 0, (th, lb, e, w)


def test_device_round_trip(cb):
    for name in ("block8", "dense_mix", "power"):
        A = MATS[name]()
        for vt in ("f64", "bf16"):
            for lb in ("contiguous", "paper"):
                M = cb.CbMatrix.from_csr(A, value_type=vt, col_agg=1, th1=8, th2=40, tile_dim=8, lb_mode=lb)
                rp, ci, va = M.export_csr()
                assert np.array_equal(rp, A.row_ptr) and np.array_equal(ci, A.col_idx)
                if vt == "f64":
                    assert np.array_equal(va.view(np.uint64), A.values.view(np.uint64))
                else:
                    assert np.array_equal(va, oracle.round_bf16_bits(A.values))
                M.close()
