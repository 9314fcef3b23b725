"""GPU parity of the quad kernel (spmv_kernel = 2: four consecutive entries of one tile per lane,
codes and values loaded straight into registers) through the C ABI against the CPU oracle: every
format mix, with and without column aggregation, every row-sum mode, alpha and beta, panels shared
between work ranges, FP64 / FP32 / BF16 storage and double vectors, exact-arithmetic inputs bit
for bit, non-finite values and x, degenerate shapes, the full-size workloads, and the serving loop's
batched launch over quad structures."""
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


def run(cb, A, x, alpha=1.0, beta=0.0, y0=None, vtype="f64", **opts):
    wide = vtype == "f64" or opts.get("vector_f64")
    dt = torch.float64 if wide else torch.float32
    M = cb.CbMatrix.from_csr(A, value_type=vtype, spmv_kernel=2, **opts)
    assert M.info["spmv_kernel"] == 2
    xd = torch.from_numpy(np.asarray(x, dtype=np.float64)).to("cuda", dt)
    yd = (torch.full((A.m,), float("nan"), dtype=dt, device="cuda") if y0 is None
          else torch.from_numpy(np.asarray(y0, dtype=np.float64)).to("cuda", dt))
    M.spmv(xd, yd, alpha, beta)
    torch.cuda.synchronize()
    out = yd.cpu().double().numpy()
    M.close()
    return out


def check(cb, A, x, alpha=1.0, beta=0.0, y0=None, vtype="f64", label="", **opts):
    y = run(cb, A, x, alpha, beta, y0, vtype, **opts)
    ref = oracle.spmv(A, x, alpha, beta, y0, comp=True)
    scl = oracle.scale(A, x, alpha, beta, y0)
    e, viol, worst = oracle.scaled_error(y, ref, scl, TOL[vtype])
    print(f"[quad {label}] {vtype} {opts} max scaled error {e:.3e}", flush=True)
    assert viol == 0, f"{label}: {viol} rows above {TOL[vtype]} (max {e}, row {worst}: {y[worst]} vs {ref[worst]})"
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


@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16", "wide"])
@pytest.mark.parametrize("name", sorted(SMALL))
def test_quad_kernel(cb, name, vtype):
    A = SMALL[name]()
    x = matgen.vector(A.n, 14)
    y0 = matgen.vector(A.m, 5, stream=matgen.STREAM_Y0)
    vt = "f32" if vtype == "wide" else vtype
    extra = {"vector_f64": 1} if vtype == "wide" else {}
    for agg, th in ((0, (32, 128)), (1, (32, 128)), (1, (8, 40)), (0, (1, 1)), (1, (300, 300))):
        check(cb, A, x, vtype=vt, label=f"{name} agg={agg} th={th}", col_agg=agg, th1=th[0], th2=th[1], **extra)
    check(cb, A, x, 1.5, -0.5, y0, vt, label=f"{name} shared", wave_nnz=64, **extra)


@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("rr", [0, 1, 2, 3, 4])
def test_quad_row_sum_modes(cb, rr, vtype):
    for name in ("block8", "power", "dense_mix"):
        A = SMALL[name]()
        x = matgen.vector(A.n, 12)
        y0 = matgen.vector(A.m, 3, stream=matgen.STREAM_Y0)
        for agg in (0, 1):
            check(cb, A, x, vtype=vtype, label=f"{name} rr={rr}", col_agg=agg, row_reduce=rr, th1=16, th2=64)
        check(cb, A, x, 1.5, -0.5, y0, vtype, label=f"{name} rr={rr} shared", row_reduce=rr, wave_nnz=64)


@pytest.mark.parametrize("lb", ["contiguous", "none"])
def test_quad_exact_bitwise(cb, lb):
    rng = np.random.default_rng(31)
    for B in (SMALL["block8"](), SMALL["dense_mix"](), SMALL["power"](), SMALL["lap13"]()):
        A = matgen.Csr(B.m, B.n, B.row_ptr, B.col_idx, rng.integers(-64, 65, B.nnz).astype(np.float64) / 64)
        x = rng.integers(-64, 65, A.n).astype(np.float64) / 64
        ref = oracle.spmv(A, x)
        for th in ((32, 128), (8, 40), (1, 1)):
            for vt in ("f64", "bf16"):
                assert np.array_equal(run(cb, A, x, vtype=vt, lb_mode=lb, th1=th[0], th2=th[1],
                                          vector_f64=1 if vt == "bf16" else 0), ref), (lb, th, vt)


def test_quad_nonfinite_and_degenerate(cb):
    # Inf / NaN in x and in the values, explicit zeros: the plain product's rules (a zero-filled
    # Dense slot never meets x)
    rng = np.random.default_rng(5)
    D = np.where(rng.random((50, 70)) < 0.6, rng.uniform(-1, 1, (50, 70)), 0.0)
    D[3, 5] = np.inf
    D[7, 9] = np.nan
    keep = D != 0
    keep[10, 10] = True  # explicit zero
    A = matgen.from_dense(D, keep_zeros_mask=keep)
    x = matgen.vector(A.n, 2)
    x[11] = np.inf
    x[40] = np.nan
    for th in ((32, 128), (1, 1), (300, 300)):
        y = run(cb, A, x, th1=th[0], th2=th[1], col_agg=0)
        ref = oracle.spmv(A, x)
        e, viol, _ = oracle.scaled_error(y, ref, oracle.scale(A, x), 1e-12)
        assert viol == 0, (th, e)
    # empty matrix, empty rows and panels, a single entry
    for A in (matgen.random_csr(0, 5, 0.5, 1), matgen.random_csr(40, 0, 0.5, 1), matgen.random_csr(100, 100, 0.0, 1),
              matgen.from_dense(np.eye(1))):
        if A.m == 0:
            continue
        x = np.ones(A.n)
        y = run(cb, A, x)
        assert np.array_equal(y, oracle.spmv(A, x))


def test_quad_graph_replays(cb):
    """The quad kernel captured in a HIP graph and replayed with eager work between replays."""
    A = SMALL["power"]()
    x = matgen.vector(A.n, 3)
    M = cb.CbMatrix.from_csr(A, spmv_kernel=2, wave_nnz=64)
    xd = torch.from_numpy(x).to("cuda")
    yd = torch.zeros(A.m, dtype=torch.float64, device="cuda")
    ref = oracle.spmv(A, x, comp=True)
    scl = oracle.scale(A, x)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        M.spmv(xd, yd, stream=s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            M.spmv(xd, yd, stream=s)
    for rep in range(4):
        yd.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        e, viol, _ = oracle.scaled_error(yd.cpu().numpy(), ref, scl, 1e-12)
        assert viol == 0, (rep, e)
    M.close()


@pytest.mark.timeout(600)
def test_quad_full_size(cb):
    """The benchmark matrices at full size: block 100^3 x 3 in FP64 / FP32 / BF16 and the 192^3
    Poisson operator on every row, the power-law matrix on sampled rows."""
    block = matgen.block_3d(100, 3, 10.0, seed=1)
    x = matgen.vector(block.n, 1)
    ref = oracle.spmv(block, x, comp=True)
    scl = oracle.scale(block, x)
    for vt in ("f64", "f32", "bf16"):
        y = run(cb, block, x, vtype=vt)
        e, viol, _ = oracle.scaled_error(y, ref, scl, TOL[vt])
        print(f"[quad block3d {vt}] max scaled error {e:.3e}", flush=True)
        assert viol == 0
    del block, ref, scl
    P = matgen.poisson_3d(192)
    x = matgen.vector(P.n, 1)
    for agg in (-1, 0):
        y = run(cb, P, x, col_agg=agg)
        e, viol, _ = oracle.scaled_error(y, oracle.spmv(P, x, comp=True), oracle.scale(P, x), 1e-12)
        print(f"[quad poisson192 agg={agg}] max scaled error {e:.3e}", flush=True)
        assert viol == 0
    del P
    Pl = matgen.power_law(4_000_000, seed=2)
    x = matgen.vector(Pl.n, 1)
    y = run(cb, Pl, x)
    lens = np.diff(Pl.row_ptr)
    rows = np.unique(np.concatenate([np.argsort(lens)[-64:], np.random.default_rng(3).choice(Pl.m, 20000,
                                                                                             replace=False)]))
    starts, ends = Pl.row_ptr[rows], Pl.row_ptr[rows + 1]
    idx = np.concatenate([np.arange(a, b) for a, b in zip(starts, ends)])
    sub = matgen.Csr(rows.size, Pl.n, np.concatenate([[0], np.cumsum(ends - starts)]).astype(np.int64),
                     Pl.col_idx[idx], Pl.values[idx])
    e, viol, _ = oracle.scaled_error(y[rows], oracle.spmv(sub, x, comp=True), oracle.scale(sub, x), 1e-12)
    print(f"[quad powerlaw 4M] max scaled error {e:.3e} over {rows.size} rows", flush=True)
    assert viol == 0


def test_quad_serving_batches(cb):
    """CG solves served in one batched launch over quad structures (and mixed with streaming-kernel
    structures) match the same solves run alone with cb_cg."""
    mats = [matgen.poisson_3d(s) for s in (10, 14, 17)]
    handles = [cb.CbMatrix.from_csr(A, spmv_kernel=2 if i != 1 else 0) for i, A in enumerate(mats)]
    S = cb.CbServer(max_active=8, arena_bytes=1 << 28)
    ids = [S.add_matrix(M) for M in handles]
    bs = [matgen.vector(A.n, 40 + i) for i, A in enumerate(mats)]
    outs = [np.zeros(A.n) for A in mats]
    tickets = [S.submit_cg(ids[i], bs[i], outs[i], rtol=1e-10, max_iter=2000) for i in range(len(mats))]
    resp = [S.wait(t) for t in tickets]
    S.close()
    for i, A in enumerate(mats):
        assert resp[i]["converged"], resp[i]
        xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        handles[i].cg(torch.from_numpy(bs[i]).to("cuda"), xd, rtol=1e-10, check_every=8, max_iter=2000)
        alone = xd.cpu().numpy()
        d = np.abs(outs[i] - alone).max() / np.abs(alone).max()
        print(f"[quad serving] matrix {i}: served vs alone {d:.3e}", flush=True)
        assert d <= 1e-8
    for M in handles:
        M.close()
