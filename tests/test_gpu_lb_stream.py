"""GPU parity of Algorithm 2's groups streamed (lb_mode paper_stream: the packed tiles re-laid in
group order, the quad kernel in scatter form, every tile's rows added into y with atomics after a
y <- beta*y pre-pass; SpMM through the tile-at-a-time kernel of Algorithm 2's order): every value
type, format mix, aggregation setting and row-sum mode against the oracle, alpha/beta special
cases, exact inputs bit for bit, and the full-size 3D block matrix row by row."""
import numpy as np
import pytest

import oracle
from paper_2605_18515_amd import matgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2}
LB = "paper_stream"


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2605_18515_amd import cbspmv

    torch.cuda.init()
    return cbspmv


MATS = {
    "lap64": lambda: matgen.laplacian_2d(64),
    "block8": lambda: matgen.block_3d(8, seed=5),
    "poisson10": lambda: matgen.poisson_3d(10),
    "power": lambda: matgen.power_law(5000, seed=3, max_len=2000, window=400),
    "rect": lambda: matgen.random_csr(301, 517, 0.03, 6),
    "dense_mix": lambda: matgen.from_dense(
        np.where(np.random.default_rng(1).random((170, 190)) < np.repeat([0.95, 0.4, 0.05], [64, 60, 46])[:, None],
                 np.random.default_rng(2).uniform(-1, 1, (170, 190)), 0.0)),
}


def run_spmv(cb, A, x, alpha=1.0, beta=0.0, y0=None, vtype="f64", **opts):
    dt = torch.float64 if vtype == "f64" or opts.get("vector_f64") else torch.float32
    M = cb.CbMatrix.from_csr(A, value_type=vtype, lb_mode=LB, **opts)
    assert M.info["lb_mode"] == cb.CB_LB_PAPER_STREAM and M.info["spmv_kernel"] == 2
    xd = torch.from_numpy(np.asarray(x, dtype=np.float64)).to("cuda", dt)
    yd = (torch.full((A.m,), float("nan"), dtype=dt, device="cuda") if y0 is None else
          torch.from_numpy(np.asarray(y0, dtype=np.float64)).to("cuda", dt))
    M.spmv(xd, yd, alpha, beta)
    torch.cuda.synchronize()
    out = yd.cpu().double().numpy()
    M.close()
    return out


def check(cb, A, x, alpha=1.0, beta=0.0, y0=None, vtype="f64", label="", **opts):
    y = run_spmv(cb, A, x, alpha, beta, y0, vtype, **opts)
    ref = oracle.spmv(A, x, alpha, beta, y0, comp=True)
    e, viol, worst = oracle.scaled_error(y, ref, oracle.scale(A, x, alpha, beta, y0), TOL[vtype])
    print(f"[{label}] {vtype} {opts} max scaled error {e:.3e}")
    assert viol == 0, f"{label}: {viol} rows above {TOL[vtype]} (max {e}, row {worst}: {y[worst]} vs {ref[worst]})"
    return y


@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("name", sorted(MATS))
def test_streamed_algorithm2_spmv(cb, name, vtype):
    A = MATS[name]()
    x = matgen.vector(A.n, 7)
    y0 = matgen.vector(A.m, 2, stream=matgen.STREAM_Y0)
    for agg in (-1, 0, 1):
        check(cb, A, x, vtype=vtype, label=f"{name} agg={agg}", col_agg=agg)
        check(cb, A, x, 1.5, -0.5, y0, vtype, label=f"{name} agg={agg} short", col_agg=agg, wave_nnz=64)
    for th in ((8, 40), (1, 1), (300, 300)):
        check(cb, A, x, vtype=vtype, label=f"{name} th={th}", th1=th[0], th2=th[1], quantum_tiles=3)


@pytest.mark.parametrize("rr", [0, 2, 3, 4])
@pytest.mark.parametrize("vtype", ["f64", "f32"])
def test_streamed_algorithm2_row_sums(cb, rr, vtype):
    for name in ("block8", "power", "dense_mix"):
        A = MATS[name]()
        x = matgen.vector(A.n, 11)
        check(cb, A, x, vtype=vtype, label=f"{name} rr={rr}", row_reduce=rr, th1=16, th2=64)
        check(cb, A, x, vtype=vtype, label=f"{name} rr={rr} wide", row_reduce=rr, vector_f64=1) \
            if vtype != "f64" else None


def test_streamed_algorithm2_alpha_beta_and_exact(cb):
    A = MATS["power"]()
    x = matgen.vector(A.n, 1)
    y0 = matgen.vector(A.m, 2, stream=matgen.STREAM_Y0)
    check(cb, A, x, 2.5, -0.75, y0, label="ab")
    y = check(cb, A, x, 0.0, 0.5, y0, label="alpha0")
    assert np.array_equal(y, 0.5 * y0)
    y = check(cb, A, x, 1.0, 0.0, np.full(A.m, np.nan), label="beta0-nan")
    assert np.isfinite(y).all()
    for name, B in [("dyadic", matgen.random_csr(500, 700, 0.04, 3, values="dyadic")),
                    ("lap", matgen.laplacian_2d(40)), ("poisson", matgen.poisson_3d(10))]:
        xd = matgen.vector(B.n, 4, dyadic=True)
        ref = oracle.spmv(B, xd)
        for agg in (0, 1):
            for th in ((32, 128), (4, 20)):
                yb = run_spmv(cb, B, xd, col_agg=agg, th1=th[0], th2=th[1], wave_nnz=64)
                assert np.array_equal(yb.view(np.uint64), ref.view(np.uint64)), (name, agg, th)


@pytest.mark.parametrize("k", [1, 5, 16, 33])
def test_streamed_algorithm2_spmm(cb, k):
    A = MATS["dense_mix"]() if k % 2 else MATS["block8"]()
    X = matgen.rhs(A.n, k, k + 3)
    Y0 = matgen.rhs(A.m, k, k + 60)
    for vtype in ("f64", "f32"):
        dt = torch.float64 if vtype == "f64" else torch.float32
        M = cb.CbMatrix.from_csr(A, value_type=vtype, lb_mode=LB, th1=8, th2=40)
        Xd = torch.from_numpy(X).to("cuda", dt)
        Yd = torch.from_numpy(Y0).to("cuda", dt)
        M.spmm(Xd, Yd, 1.5, -0.5)
        torch.cuda.synchronize()
        Y = Yd.cpu().double().numpy()
        M.close()
        e, viol, _ = oracle.scaled_error(Y.ravel(), oracle.spmm(A, X, 1.5, -0.5, Y0, comp=True).ravel(),
                                         oracle.spmm_scale(A, X, 1.5, -0.5, Y0).ravel(), TOL[vtype])
        assert viol == 0, (k, vtype, e)


@pytest.mark.slow
def test_streamed_algorithm2_full_block(cb):
    """The benchmark's 3D block matrix (62,460,000 entries) under Algorithm 2's streamed groups: every
    row in FP64 against the oracle."""
    A = matgen.block_3d(100, 3, 10.0, seed=1)
    x = matgen.vector(A.n, 1)
    y = run_spmv(cb, A, x)
    e, viol, worst = oracle.scaled_error(y, oracle.spmv(A, x, comp=True), oracle.scale(A, x), 1e-12)
    print(f"block 100^3 x 3 paper_stream: max scaled error {e:.3e}")
    assert viol == 0, (e, worst)
