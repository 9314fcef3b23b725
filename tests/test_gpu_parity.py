"""GPU parity: the HIP path through the C ABI against the CPU oracle on the same
seeded inputs.  FP64 storage must satisfy |y - y_ref| <= 1e-12 (|alpha||A||x| +
|beta||y0|) row by row; FP32 storage 1e-5; BF16 storage 1e-2 (all against the
FP64 oracle on the original values); exact-arithmetic inputs must match bit for
bit whatever the summation order."""
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


def run_spmv(cb, A, x, alpha=1.0, beta=0.0, y0=None, vtype="f64", **opts):
    dt = torch.float64 if vtype == "f64" or opts.get("vector_f64") else torch.float32
    M = cb.CbMatrix.from_csr(A, value_type=vtype, **opts)
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


def lowp(v, vtype):
    if vtype == "f32":
        return oracle.f32_values(v)
    if vtype == "bf16":
        return oracle.bf16_values(v)
    return np.asarray(v, dtype=np.float64)


def check(cb, A, x, alpha=1.0, beta=0.0, y0=None, vtype="f64", label="", **opts):
    y = run_spmv(cb, A, x, alpha, beta, y0, vtype, **opts)
    ref = oracle.spmv(A, x, alpha, beta, y0, comp=True)
    scl = oracle.scale(A, x, alpha, beta, y0)
    e, viol, worst = oracle.scaled_error(y, ref, scl, TOL[vtype])
    print(f"[{label}] {vtype} {opts} max scaled error {e:.3e}")
    assert viol == 0, f"{label}: {viol} rows above {TOL[vtype]} (max {e}, row {worst}: {y[worst]} vs {ref[worst]})"
    if vtype != "f64":
        # against the oracle on the stored (rounded) values and rounded x, alpha, beta:
        # only the FP32 accumulation remains
        xr = oracle.f32_values(x)
        y0r = None if y0 is None else oracle.f32_values(y0)
        a32, b32 = float(np.float32(alpha)), float(np.float32(beta))
        ref2 = oracle.spmv(A, xr, a32, b32, y0r, comp=True, values=lowp(A.values, vtype))
        scl2 = oracle.scale(A, xr, a32, b32, y0r, values=lowp(A.values, vtype))
        rowlen = np.diff(A.row_ptr).max() if A.m else 0
        bound = 2 * (rowlen + 4) * 2.0 ** -24
        e2, v2, _ = oracle.scaled_error(y, ref2, scl2, bound)
        assert v2 == 0, f"{label}: FP32 accumulation error {e2} above {bound}"
    return y


SMALL = {
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


@pytest.mark.parametrize("name", sorted(SMALL))
@pytest.mark.parametrize("lb", ["contiguous", "paper", "none"])
@pytest.mark.parametrize("col_agg", [-1, 0, 1])
def test_spmv_f64(cb, name, lb, col_agg):
    A = SMALL[name]()
    x = matgen.vector(A.n, 7)
    check(cb, A, x, label=name, lb_mode=lb, col_agg=col_agg)
    # short work ranges: these matrices then span many ranges, with panels shared between them
    check(cb, A, x, label=f"{name} short ranges", lb_mode=lb, col_agg=col_agg, wave_nnz=64)


@pytest.mark.parametrize("name", ["dense_mix", "power", "block8"])
@pytest.mark.parametrize("th", [(32, 128), (8, 40), (1, 1), (300, 300)])
def test_spmv_formats(cb, name, th):
    A = SMALL[name]()
    x = matgen.vector(A.n, 8)
    for agg in (0, 1):
        check(cb, A, x, label=f"{name} th={th}", col_agg=agg, th1=th[0], th2=th[1])


@pytest.mark.parametrize("vtype", ["f32", "bf16"])
@pytest.mark.parametrize("name", ["block8", "dense_mix", "lap64", "rect"])
def test_spmv_low_precision(cb, name, vtype):
    A = SMALL[name]()
    x = matgen.vector(A.n, 9)
    for agg in (0, 1):
        check(cb, A, x, vtype=vtype, label=name, col_agg=agg, th1=16, th2=64)


@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("rr", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("name", ["block8", "power", "lap64", "dense_mix", "rect"])
def test_row_reduce_modes(cb, name, rr, vtype):
    """Every way the streaming kernel sums rows (LDS atomics, DPP segmented scan, FP64 atomics,
    and the atomics into two accumulator copies), with and without column aggregation, and with
    several work ranges sharing panels."""
    A = SMALL[name]()
    x = matgen.vector(A.n, 12)
    y0 = matgen.vector(A.m, 3, stream=matgen.STREAM_Y0)
    for agg in (0, 1):
        check(cb, A, x, vtype=vtype, label=f"{name} rr={rr}", col_agg=agg, row_reduce=rr, th1=16, th2=64)
    check(cb, A, x, 1.5, -0.5, y0, vtype, label=f"{name} rr={rr} shared", row_reduce=rr, wave_nnz=64)


@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16", "wide"])
@pytest.mark.parametrize("name", ["block8", "power", "lap64", "dense_mix", "rect", "wide", "poisson12"])
def test_rows_kernel(cb, name, vtype):
    """The rows-per-lane kernel (spmv_kernel = 1): every format mix, with and without aggregation,
    alpha and beta, and panels shared between work ranges."""
    A = SMALL[name]()
    x = matgen.vector(A.n, 14)
    y0 = matgen.vector(A.m, 5, stream=matgen.STREAM_Y0)
    vt = "f32" if vtype == "wide" else vtype
    extra = {"vector_f64": 1} if vtype == "wide" else {}
    for agg, th in ((0, (32, 128)), (1, (32, 128)), (1, (8, 40)), (0, (1, 1)), (1, (300, 300))):
        check(cb, A, x, vtype=vt, label=f"{name} rows agg={agg} th={th}", col_agg=agg, th1=th[0], th2=th[1],
              spmv_kernel=1, **extra)
    check(cb, A, x, 1.5, -0.5, y0, vt, label=f"{name} rows shared", spmv_kernel=1, wave_nnz=64, **extra)


def test_rows_kernel_exact_bitwise(cb):
    rng = np.random.default_rng(29)
    for B in (SMALL["block8"](), SMALL["dense_mix"](), SMALL["power"]()):
        A = matgen.Csr(B.m, B.n, B.row_ptr, B.col_idx, rng.integers(-64, 65, B.nnz).astype(np.float64) / 64)
        x = rng.integers(-64, 65, A.n).astype(np.float64) / 64
        ref = oracle.spmv(A, x)
        for th in ((32, 128), (8, 40)):
            assert np.array_equal(run_spmv(cb, A, x, spmv_kernel=1, th1=th[0], th2=th[1]), ref)


def rounded(A, vtype):
    return matgen.Csr(A.m, A.n, A.row_ptr, A.col_idx, lowp(A.values, vtype))


@pytest.mark.parametrize("vtype", ["f32", "bf16"])
@pytest.mark.parametrize("rr", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("name", ["block8", "power", "lap64", "dense_mix", "rect"])
def test_wide_vectors(cb, name, rr, vtype):
    """FP32/BF16 storage with double x and y: FP64 arithmetic on the widened stored values, so the
    result is the FP64 oracle's on the rounded values to 1e-12, and the FP64 matrix's to the
    storage precision's tolerance."""
    A = SMALL[name]()
    Ar = rounded(A, vtype)
    x = matgen.vector(A.n, 13)
    y0 = matgen.vector(A.m, 4, stream=matgen.STREAM_Y0)
    for lb, agg in (("contiguous", 0), ("contiguous", 1), ("paper", -1)):
        for al, be, yy in ((1.0, 0.0, None), (1.5, -0.5, y0)):
            y = run_spmv(cb, A, x, al, be, yy, vtype, vector_f64=1, lb_mode=lb, col_agg=agg, row_reduce=rr,
                         th1=16, th2=64)
            e, viol, w = oracle.scaled_error(y, oracle.spmv(Ar, x, al, be, yy, comp=True),
                                             oracle.scale(Ar, x, al, be, yy), 1e-12)
            print(f"[{name} {vtype} wide rr={rr} {lb} agg={agg}] max scaled error vs rounded values {e:.3e}")
            assert viol == 0, (lb, agg, e, w)
            e2, v2, _ = oracle.scaled_error(y, oracle.spmv(A, x, al, be, yy, comp=True),
                                            oracle.scale(A, x, al, be, yy), TOL[vtype])
            assert v2 == 0, (lb, agg, e2)


@pytest.mark.parametrize("k", [1, 8, 17, 32])
@pytest.mark.parametrize("vtype", ["f32", "bf16"])
def test_wide_vectors_spmm(cb, k, vtype):
    A = SMALL["dense_mix"]() if k % 2 else SMALL["block8"]()
    Ar = rounded(A, vtype)
    X = matgen.rhs(A.n, k, k + 3)
    Y0 = matgen.rhs(A.m, k, k + 60)
    for lb, agg in (("contiguous", -1), ("paper", 0), ("contiguous", 1)):
        Y = run_spmm(cb, A, X, 1.5, -0.5, Y0, vtype, ld_pad=2, vector_f64=1, lb_mode=lb, col_agg=agg, th1=8, th2=40)
        e, viol, _ = oracle.scaled_error(Y, oracle.spmm(Ar, X, 1.5, -0.5, Y0, comp=True),
                                         oracle.spmm_scale(Ar, X, 1.5, -0.5, Y0), 1e-12)
        print(f"spmm wide k={k} {vtype} {lb} agg={agg} max scaled error {e:.3e}")
        assert viol == 0, (k, vtype, lb, e)


def test_wide_vectors_exact_bitwise(cb):
    # values and x with at most 7 significant bits: exact in BF16, every product and sum exact in FP64
    rng = np.random.default_rng(23)
    B = SMALL["power"]()
    A = matgen.Csr(B.m, B.n, B.row_ptr, B.col_idx, rng.integers(-64, 65, B.nnz).astype(np.float64) / 64)
    x = rng.integers(-64, 65, A.n).astype(np.float64) / 64
    ref = oracle.spmv(A, x)
    for vt in ("f32", "bf16"):
        for rr in (0, 1, 2, 3, 4):
            assert np.array_equal(run_spmv(cb, A, x, vtype=vt, vector_f64=1, row_reduce=rr), ref), (vt, rr)


def test_row_reduce_exact_bitwise(cb):
    rng = np.random.default_rng(21)
    B = SMALL["block8"]()
    A = matgen.Csr(B.m, B.n, B.row_ptr, B.col_idx, rng.integers(-64, 65, B.nnz).astype(np.float64) / 64)
    x = rng.integers(-64, 65, A.n).astype(np.float64) / 64
    ref = oracle.spmv(A, x)
    for rr in (0, 1, 2, 3, 4):
        assert np.array_equal(run_spmv(cb, A, x, row_reduce=rr), ref)


@pytest.mark.parametrize("vtype", ["f64", "f32"])
def test_alpha_beta(cb, vtype):
    A = SMALL["power"]()
    x = matgen.vector(A.n, 1)
    y0 = matgen.vector(A.m, 2, stream=matgen.STREAM_Y0)
    for lb in ("contiguous", "paper"):
        check(cb, A, x, 2.5, -0.75, y0, vtype, label="ab", lb_mode=lb)
        check(cb, A, x, 0.0, 0.5, y0, vtype, label="alpha0", lb_mode=lb)
        y = check(cb, A, x, 1.0, 0.0, np.full(A.m, np.nan), vtype, label="beta0-nan", lb_mode=lb)
        assert np.isfinite(y).all()


@pytest.mark.parametrize("lb", ["contiguous", "paper", "none"])
def test_exact_arithmetic_bitwise(cb, lb):
    for name, A in [("dyadic", matgen.random_csr(500, 700, 0.04, 3, values="dyadic")),
                    ("lap", matgen.laplacian_2d(40)), ("poisson", matgen.poisson_3d(10))]:
        x = matgen.vector(A.n, 4, dyadic=True)
        ref = oracle.spmv(A, x)
        for agg in (0, 1):
            for th in ((32, 128), (4, 20)):
                y = run_spmv(cb, A, x, lb_mode=lb, col_agg=agg, th1=th[0], th2=th[1], wave_nnz=64)
                assert np.array_equal(y.view(np.uint64), ref.view(np.uint64)), (name, agg, th)


def test_identity_and_permutation_bitwise(cb):
    x = matgen.vector(1000, 3)
    I = matgen.identity(1000)
    assert np.array_equal(run_spmv(cb, I, x).view(np.uint64), x.view(np.uint64))
    P, pi = matgen.permutation(1000, 3)
    for agg in (0, 1):
        assert np.array_equal(run_spmv(cb, P, x, col_agg=agg).view(np.uint64), x[pi].view(np.uint64))


def test_laplacian_closed_form(cb):
    A = matgen.laplacian_2d(64)
    r = np.arange(64 * 64)
    i, j = r % 64, r // 64
    y = run_spmv(cb, A, np.ones(64 * 64))
    assert np.array_equal(y, ((i == 0).astype(int) + (i == 63) + (j == 0) + (j == 63)).astype(float))


def test_empty_and_degenerate(cb):
    y0 = np.arange(40, dtype=np.float64)
    A = matgen.Csr(40, 30, np.zeros(41, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert np.array_equal(run_spmv(cb, A, np.ones(30), 1.0, 0.5, y0), 0.5 * y0)
    assert np.array_equal(run_spmv(cb, A, np.ones(30), 1.0, 0.0, np.full(40, np.nan)), np.zeros(40))
    B = matgen.Csr(0, 5, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert run_spmv(cb, B, np.ones(5)).size == 0
    D = np.zeros((100, 60)); D[3, 5] = 1.0; D[70, 59] = 2.0; D[99, 0] = 3.0
    check(cb, matgen.from_dense(D), matgen.vector(60, 1), 1.0, 2.0, np.ones(100), label="empty panels")


def test_nonfinite_x_and_values(cb):
    rng = np.random.default_rng(5)
    A = SMALL["dense_mix"]()
    vals = A.values.copy()
    vals[rng.integers(0, A.nnz, 20)] = np.nan
    vals[rng.integers(0, A.nnz, 20)] = np.inf
    B = matgen.Csr(A.m, A.n, A.row_ptr, A.col_idx, vals)
    x = matgen.vector(A.n, 5)
    x[rng.integers(0, A.n, 5)] = np.inf
    for th in ((32, 128), (4, 16)):  # dense tiles must not multiply their zero fill with Inf
        check(cb, B, x, label="nonfinite", col_agg=0, th1=th[0], th2=th[1])
        check(cb, B, x, label="nonfinite", col_agg=1, th1=th[0], th2=th[1])


def run_spmm(cb, A, X, alpha, beta, Y0, vtype="f64", ld_pad=0, **opts):
    dt = torch.float64 if vtype == "f64" or opts.get("vector_f64") else torch.float32
    k = X.shape[1]
    M = cb.CbMatrix.from_csr(A, value_type=vtype, **opts)
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


@pytest.mark.parametrize("k", [1, 2, 3, 8, 17, 32, 40])
@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
def test_spmm(cb, k, vtype):
    A = SMALL["dense_mix"]() if k % 2 else SMALL["block8"]()
    X = matgen.rhs(A.n, k, k)
    Y0 = matgen.rhs(A.m, k, k + 50)
    for lb, agg, th, wn in (("contiguous", -1, (32, 128), 0), ("paper", 0, (8, 40), 0), ("contiguous", 1, (8, 40), 0),
                            ("contiguous", -1, (32, 128), 64), ("none", 1, (8, 40), 64)):
        Y = run_spmm(cb, A, X, 1.5, -0.5, Y0, vtype, ld_pad=3, lb_mode=lb, col_agg=agg, th1=th[0], th2=th[1],
                     wave_nnz=wn)
        ref = oracle.spmm(A, X, 1.5, -0.5, Y0, comp=True)
        scl = oracle.spmm_scale(A, X, 1.5, -0.5, Y0)
        e, viol, _ = oracle.scaled_error(Y, ref, scl, TOL[vtype])
        print(f"spmm k={k} {vtype} {lb} agg={agg} max scaled error {e:.3e}")
        assert viol == 0, (k, vtype, lb, e)


def test_spmm_exact_bitwise(cb):
    A = matgen.random_csr(300, 280, 0.06, 11, values="dyadic")
    X = np.random.default_rng(1).integers(-64, 65, (280, 8)).astype(np.float64) / 64
    ref = oracle.spmm(A, X)
    for th in ((32, 128), (2, 10)):
        Y = run_spmm(cb, A, X, 1.0, 0.0, np.zeros((300, 8)), col_agg=0, th1=th[0], th2=th[1])
        assert np.array_equal(Y.view(np.uint64), ref.view(np.uint64))


def test_device_round_trip(cb):
    for name in ("block8", "dense_mix", "power"):
        A = SMALL[name]()
        for vt in ("f64", "bf16"):
            M = cb.CbMatrix.from_csr(A, value_type=vt, col_agg=1, th1=8, th2=40)
            rp, ci, va = M.export_csr()
            assert M.info["on_device"] == 1
            assert np.array_equal(rp, A.row_ptr) and np.array_equal(ci, A.col_idx)
            if vt == "f64":
                assert np.array_equal(va.view(np.uint64), A.values.view(np.uint64))
            else:
                assert np.array_equal(va, oracle.round_bf16_bits(A.values))
            M.close()


def test_repeated_calls_and_streams(cb):
    A = SMALL["power"]()
    x = matgen.vector(A.n, 1)
    ref = oracle.spmv(A, x, comp=True)
    scl = oracle.scale(A, x)
    M = cb.CbMatrix.from_csr(A, lb_mode="paper")
    xd = torch.from_numpy(x).cuda()
    s = torch.cuda.Stream()
    ys = []
    with torch.cuda.stream(s):
        for _ in range(5):
            yd = torch.empty(A.m, dtype=torch.float64, device="cuda")
            M.spmv(xd, yd)
            ys.append(yd)
    torch.cuda.synchronize()
    for yd in ys:
        assert oracle.scaled_error(yd.cpu().numpy(), ref, scl, 1e-12)[1] == 0
    M.close()


@pytest.mark.parametrize("lb,wn", [("contiguous", 64), ("paper", 0)])
def test_graph_replays(cb, lb, wn):
    """cb_spmv and cb_spmm captured in one HIP graph (with shared panels, so the y <- beta y pre-pass is
    captured too) and replayed several times, with eager work and synchronisations between the
    replays: every replay meets the oracle."""
    A = SMALL["power"]()
    k = 8
    x, y0 = matgen.vector(A.n, 2), matgen.vector(A.m, 5, stream=matgen.STREAM_Y0)
    X, Y0 = matgen.rhs(A.n, k, 3), matgen.rhs(A.m, k, 4)
    M = cb.CbMatrix.from_csr(A, lb_mode=lb, wave_nnz=wn)
    if lb == "contiguous":
        assert M.info["shared_panels"] > 0
    xd, y0d = torch.from_numpy(x).cuda(), torch.from_numpy(y0).cuda()
    Xd, Y0d = torch.from_numpy(X).cuda(), torch.from_numpy(Y0).cuda()
    yd, Yd = torch.empty_like(y0d), torch.empty_like(Y0d)
    ref = oracle.spmv(A, x, 1.5, -0.5, y0, comp=True)
    scl = oracle.scale(A, x, 1.5, -0.5, y0)
    refm = oracle.spmm(A, X, 1.5, -0.5, Y0, comp=True)
    sclm = oracle.spmm_scale(A, X, 1.5, -0.5, Y0)

    def step():
        yd.copy_(y0d)
        M.spmv(xd, yd, 1.5, -0.5)
        Yd.copy_(Y0d)
        M.spmm(Xd, Yd, 1.5, -0.5)

    step()  # eager: code objects loaded before the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(4):
        yd.fill_(float("nan"))
        Yd.fill_(7.0)
        M.spmv(xd, torch.empty_like(yd))  # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert oracle.scaled_error(yd.cpu().numpy(), ref, scl, 1e-12)[1] == 0, rep
        assert oracle.scaled_error(Yd.cpu().numpy(), refm, sclm, 1e-12)[1] == 0, rep
    M.close()


def test_copy_probe(cb):
    n = 1 << 22
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    cb.cb_copy_probe(src, dst, n * 8)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_read_probe(cb):
    """Reads without writing: a zero buffer folds to 0, so the sink keeps its contents; a ragged
    size (not a multiple of the four-load step) runs the tail loop."""
    for n16 in (1, 4096 * 256 + 3, 1 << 22):
        src = torch.zeros(2 * n16, dtype=torch.float64, device="cuda")
        sink = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
        cb.cb_read_probe(src, n16 * 16, sink)
        torch.cuda.synchronize()
        assert sink.tolist() == [7.0, 7.0]


@pytest.mark.parametrize("vtype", ["f64", "f32"])
def test_spmm_dense_tiles_with_nonfinite_x(cb, vtype):
    """Dense tiles go to the matrix cores unless the staged X rows hold Inf/NaN:
    a zero-filled slot must not turn 0 * Inf into NaN."""
    A = SMALL["dense_mix"]()
    k = 16
    X = matgen.rhs(A.n, k, 3)
    X[5, 3] = np.inf
    X[40, 0] = -np.inf
    X[77, 9] = np.nan
    Y0 = np.zeros((A.m, k))
    for th in ((8, 40), (32, 128)):
        Y = run_spmm(cb, A, X, 1.0, 0.0, Y0, vtype, col_agg=0, th1=th[0], th2=th[1])
        ref = oracle.spmm(A, X, comp=True)
        e, viol, w = oracle.scaled_error(Y, ref, oracle.spmm_scale(A, X), TOL[vtype])
        assert viol == 0, (th, e, w)


@pytest.mark.parametrize("opts", [{"spmv_kernel": 0}, {"spmv_kernel": 2}, {"lb_mode": "paper_stream"},
                                  {"spmv_kernel": 0, "tile_dim": 8}, {"spmv_kernel": 2, "tile_dim": 8},
                                  {"spmv_kernel": 0, "lb_mode": "none"}])
def test_compressed_columns_match_four_byte_columns(cb, opts):
    """The 2-byte column offsets (cols16) compute what the 4-byte columns compute, in both streaming
    kernels, Algorithm 2's streamed order and both tile sizes, FP64 and FP32 values, with short
    ranges (many partial gathers at a range's end): bit for bit on exact inputs (dyadic values and x:
    every order of the row sums gives the same result; on other inputs the order of the LDS atomics
    varies from run to run), and within the tolerance of the oracle on the generators' values."""
    from test_convert import _poisson_box

    B = matgen.block_3d(10, seed=2)
    Bd = matgen.Csr(B.m, B.n, B.row_ptr, B.col_idx,
                    np.random.default_rng(5).integers(-16, 17, B.nnz).astype(np.float64) / 16)
    # planes 40,000 rows apart: the quad kernel's batches span more than 65,535 columns (per-tile bases)
    box = _poisson_box(200, 200, 3)
    for A in (B, Bd, matgen.poisson_3d(20), matgen.laplacian_2d(64), box):
        exact = A is not B
        x = matgen.vector(A.n, 4, dyadic=exact)
        for vt in ("f64", "f32"):
            # the box with the automatic ranges: several panels per range, so its quad batches span
            # its planes
            kw = dict(col_agg=1, wave_nnz=0 if A is box else 64, cols16=1, **opts)
            M = cb.CbMatrix.from_csr(A, value_type=vt, **kw)
            # the quad kernel: per-batch bases where a batch's columns span less than 65,536 (all but
            # the box), else per-tile bases, as the streaming kernel
            quad = opts.get("spmv_kernel") == 2 or opts.get("lb_mode") == "paper_stream"
            want = 2 if quad and A is not box else 1
            assert M.info["col_agg"] == 1 and M.info["cols16"] == want, (M.info["cols16"], want)
            M.close()
            y16 = run_spmv(cb, A, x, vtype=vt, **kw)
            if exact:
                y32 = run_spmv(cb, A, x, vtype=vt, **dict(kw, cols16=-1))
                assert np.array_equal(y16, y32), (A.n, vt, opts)
            ref = oracle.spmv(A, x, comp=True)
            e, viol, _ = oracle.scaled_error(y16, ref, oracle.scale(A, x), TOL[vt])
            assert viol == 0, (A.n, vt, opts, e)


@pytest.mark.parametrize("chunk", [0, 1, 3, 16, 1000])
def test_xcd_mapping_leaves_results_unchanged(cb, chunk):
    """Every workgroup-to-range mapping computes the same product: bit for bit on exact inputs
    (SpMV in both natural-order kernels and Algorithm 2's streamed order, and SpMM), within the
    tolerance otherwise."""
    A = matgen.random_csr(900, 1100, 0.02, 7, values="dyadic")
    x = matgen.vector(A.n, 3, dyadic=True)
    ref = oracle.spmv(A, x)
    for opts in ({"spmv_kernel": 0}, {"spmv_kernel": 2}, {"lb_mode": "paper_stream"}, {"lb_mode": "paper"}):
        y = run_spmv(cb, A, x, xcd_chunk=chunk, wave_nnz=64, **opts)
        assert np.array_equal(y.view(np.uint64), ref.view(np.uint64)), (chunk, opts)
    B = SMALL["block8"]()
    xb = matgen.vector(B.n, 5)
    check(cb, B, xb, label=f"block8 chunk={chunk}", xcd_chunk=chunk)
    X = np.stack([matgen.vector(A.n, 10 + j, dyadic=True) for j in range(8)], 1)
    M = cb.CbMatrix.from_csr(A, xcd_chunk=chunk, wave_nnz=64)
    Yd = torch.empty((A.m, 8), dtype=torch.float64, device="cuda")
    M.spmm(torch.from_numpy(X).to("cuda"), Yd)
    torch.cuda.synchronize()
    M.close()
    assert np.array_equal(Yd.cpu().numpy(), oracle.spmm(A, X))
