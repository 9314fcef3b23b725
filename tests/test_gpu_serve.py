"""GPU tests of the serving loop (cb_server_*): SpMM requests against the oracle and against
the direct product, CG solves alone and in a mix of other solves and SpMM requests (the same
result, iteration for iteration), graph replay against plain launches, admission under a small
memory arena, the iteration cap, breakdown on a negative definite matrix, and the statistics."""
import numpy as np
import pytest

import oracle
from oracle import solvers
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


def spd_matrices():
    """SPD operators of uneven sizes: 2D Laplacians, 3D Poisson operators, a scaled Poisson."""
    out = [matgen.laplacian_2d(s) for s in (9, 23, 40)] + [matgen.poisson_3d(s) for s in (6, 13)]
    P = matgen.poisson_3d(10)
    s = np.random.default_rng(4).uniform(0.8, 1.25, P.n)
    out.append(matgen.Csr(P.m, P.n, P.row_ptr, P.col_idx, s[P.rows()] * P.values * s[P.col_idx]))
    return out


def general_matrices():
    return [matgen.block_3d(5, seed=1), matgen.power_law(3000, seed=2, max_len=800, window=300),
            matgen.random_csr(200, 333, 0.05, 4), matgen.laplacian_2d(17)]


def make(cb, A, vt, **opts):
    if vt == "f32w":
        return cb.CbMatrix.from_csr(A, value_type="f32", vector_f64=1, **opts)
    return cb.CbMatrix.from_csr(A, value_type=vt, **opts)


def ndt(vt):
    return np.float64 if vt in ("f64", "f32w") else np.float32


def test_spmm_requests_match_oracle_and_direct(cb):
    mats = []
    with cb.CbServer(max_active=8) as S:
        reqs = []
        rng = np.random.default_rng(5)
        for A in general_matrices():
            for vt in ("f64", "f32", "f32w"):
                M = make(cb, A, vt)
                mats.append(M)
                mid = S.add_matrix(M)
                for k in (1, 3, 16):
                    X = rng.uniform(-1, 1, (A.n, k)).astype(ndt(vt))
                    Y0 = rng.uniform(-1, 1, (A.m, k)).astype(ndt(vt))
                    Y = Y0.copy()
                    reqs.append((A, M, vt, k, X, Y0, Y, S.submit_spmm(mid, X, Y, 1.5, -0.5)))
        for A, M, vt, k, X, Y0, Y, t in reqs:
            r = S.wait(t)
            assert r["done"] == 1 and r["status"] == cb.CB_SUCCESS
            Xd = X.astype(np.float64)
            ref = oracle.spmm(A, Xd, 1.5, -0.5, Y0.astype(np.float64), comp=True)
            scl = oracle.spmm_scale(A, Xd, 1.5, -0.5, Y0.astype(np.float64))
            tol = TOL["f64"] if vt == "f64" else TOL["f32"]
            e, viol, _ = oracle.scaled_error(Y.astype(np.float64).ravel(), ref.ravel(), scl.ravel(), tol)
            assert viol == 0, (vt, k, e)
            # the same product straight through cb_spmm
            dt = torch.float64 if ndt(vt) == np.float64 else torch.float32
            Yd = torch.from_numpy(Y0).to("cuda")
            M.spmm(torch.from_numpy(X).to("cuda", dt).reshape(A.n, k), Yd.reshape(A.m, k), 1.5, -0.5)
            torch.cuda.synchronize()
            e2, viol2, _ = oracle.scaled_error(Y.astype(np.float64).ravel(), Yd.cpu().double().numpy().ravel(),
                                               scl.ravel(), 1e-13 if vt != "f32" else 1e-6)
            assert viol2 == 0, (vt, k, e2)
        st = S.stats()
        assert st["spmm_done"] == len(reqs) and st["completed"] == len(reqs) and st["rejected"] == 0
    for M in mats:
        M.close()


def run_solves(cb, specs, mix_spmm=False, **opts):
    """Submit every CG request (A, vector type, seed of b[, conversion options]) at once, with SpMM
    requests in between when mix_spmm; returns [(x, response)] in submission order."""
    mats, out = [], []
    with cb.CbServer(**opts) as S:
        ids = []
        for A, vt, _, *conv in specs:
            M = make(cb, A, vt, **(conv[0] if conv else {}))
            mats.append(M)
            ids.append(S.add_matrix(M))
        extra = []
        if mix_spmm:
            G = matgen.block_3d(6, seed=3)
            MG = cb.CbMatrix.from_csr(G)
            mats.append(MG)
            gid = S.add_matrix(MG)
        tickets = []
        for i, (A, vt, seed, *_) in enumerate(specs):
            b = matgen.vector(A.n, seed).astype(ndt(vt))
            x = np.zeros(A.n, ndt(vt))
            tickets.append((x, S.submit_cg(ids[i], b, x, rtol=1e-10 if ndt(vt) == np.float64 else 1e-5,
                                           max_iter=2000)))
            if mix_spmm:
                X = np.random.default_rng(i).uniform(-1, 1, (G.n, 4))
                Y = np.zeros((G.m, 4))
                extra.append(S.submit_spmm(gid, X, Y))
        for x, t in tickets:
            out.append((x, S.wait(t)))
        for t in extra:
            assert S.wait(t)["status"] == cb.CB_SUCCESS
        stats = S.stats()
    for M in mats:
        M.close()
    return out, stats


def test_cg_alone_and_in_a_mix_agree(cb):
    spd = spd_matrices()
    specs = [(A, vt, 30 + 3 * i + j) for i, A in enumerate(spd) for j, vt in enumerate(("f64", "f32", "f32w"))]
    alone = [run_solves(cb, [s])[0][0] for s in specs]
    mixed, stats = run_solves(cb, specs, mix_spmm=True, max_active=8)
    assert stats["active_peak"] > 1 and stats["graph_builds"] >= 2
    for (A, vt, seed), (xa, ra), (xm, rm) in zip(specs, alone, mixed):
        assert ra["status"] == rm["status"] == cb.CB_SUCCESS
        assert ra["converged"] and rm["converged"], (A.name, vt, ra, rm)
        # the same arithmetic per solve: bit for bit unless panels shared between work ranges are
        # summed with global atomics (their order varies)
        shared = cb.CbMatrix.from_csr(A, device=False, value_type="f64" if vt == "f64" else "f32").info["shared_panels"]
        if shared == 0:
            assert ra["iterations"] == rm["iterations"]
            assert np.array_equal(xa, xm), (A.name, vt, np.abs(xa - xm).max())
        else:
            assert abs(ra["iterations"] - rm["iterations"]) <= 8
            tol = 1e-8 if ndt(vt) == np.float64 else 1e-3
            assert np.abs(xa - xm).max() <= tol * np.abs(xa).max(), (A.name, vt, np.abs(xa - xm).max())
        if ndt(vt) == np.float64:
            b = matgen.vector(A.n, seed)
            Aeff = A if vt == "f64" else matgen.Csr(A.m, A.n, A.row_ptr, A.col_idx, oracle.f32_values(A.values))
            assert solvers.residual(Aeff, b, xm) <= 2e-10, (A.name, vt)


@pytest.mark.parametrize("vt,modes", [("f64", (0, 1, 3)), ("f32", (1, 2, 4))])
def test_batched_products_in_every_row_sum_mode(cb, vt, modes):
    """The batched product kernel in each row-sum mode: the automatic choice gives these operators
    the one-copy modes, so every mode is forced; one server holds the solves of all modes at once
    (one launch per mode), and each result equals the same solve served alone."""
    specs = [(A, vt, 70 + 5 * i + j, {"row_reduce": rr})
             for i, A in enumerate((matgen.poisson_3d(9), matgen.laplacian_2d(30))) for j, rr in enumerate(modes)]
    alone = [run_solves(cb, [s])[0][0] for s in specs]
    mixed, stats = run_solves(cb, specs, max_active=16)
    assert stats["active_peak"] >= 2
    for (A, _, seed, conv), (xa, ra), (xm, rm) in zip(specs, alone, mixed):
        assert ra["converged"] and rm["converged"], (A.name, conv, ra, rm)
        shared = cb.CbMatrix.from_csr(A, device=False, value_type=vt, **conv).info["shared_panels"]
        if shared == 0:
            assert ra["iterations"] == rm["iterations"] and np.array_equal(xa, xm), (A.name, conv)
        else:
            assert np.abs(xa - xm).max() <= 1e-3 * np.abs(xa).max(), (A.name, conv)
        if vt == "f64":
            assert solvers.residual(A, matgen.vector(A.n, seed), xm) <= 2e-10, (A.name, conv)


def test_graph_replay_matches_plain_launches(cb):
    specs = [(A, "f64", 40 + i) for i, A in enumerate(spd_matrices()[:4])]
    g, sg = run_solves(cb, specs, use_graph=1, max_active=4)
    p, sp = run_solves(cb, specs, use_graph=0, max_active=4)
    # a set's first period runs as plain launches, the later ones replay its graph
    assert sg["graph_builds"] >= 1 and sp["graph_builds"] == 0
    for (xg, rg), (xp, rp) in zip(g, p):
        assert rg["iterations"] == rp["iterations"] and np.array_equal(xg, xp)


def test_admission_under_a_small_arena(cb):
    A = matgen.laplacian_2d(40)  # 1600 unknowns: a solve takes 5 x 12.8 KB
    specs = [(A, "f64", 50 + i) for i in range(12)]
    res, st = run_solves(cb, specs, arena_bytes=3 * 5 * 12800 + 4096, max_active=8)
    assert all(r["converged"] for _, r in res)
    assert st["arena_peak_bytes"] <= 3 * 5 * 12800 + 4096 and st["active_peak"] <= 3
    assert max(r["queue_us"] for _, r in res) > 0
    # a request that can never fit is refused at submission
    M = cb.CbMatrix.from_csr(matgen.laplacian_2d(64))
    with cb.CbServer(arena_bytes=4096) as S:
        mid = S.add_matrix(M)
        with pytest.raises(cb.CbError) as e:
            S.submit_cg(mid, np.ones(4096), np.zeros(4096))
        assert e.value.status == cb.CB_ERROR_OUT_OF_MEMORY
        assert S.stats()["rejected"] == 1
    M.close()


def test_iteration_cap_and_breakdown(cb):
    A = matgen.poisson_3d(12)
    N = matgen.laplacian_2d(12)
    N = matgen.Csr(N.m, N.n, N.row_ptr, N.col_idx, -N.values)
    Ms = [cb.CbMatrix.from_csr(A), cb.CbMatrix.from_csr(N)]
    with cb.CbServer(check_every=4) as S:
        a, n = S.add_matrix(Ms[0]), S.add_matrix(Ms[1])
        x1, x2 = np.zeros(A.n), np.zeros(N.n)
        t1 = S.submit_cg(a, matgen.vector(A.n, 1), x1, max_iter=6)
        t2 = S.submit_cg(n, matgen.vector(N.n, 2), x2)
        r1, r2 = S.wait(t1), S.wait(t2)
    assert not r1["converged"] and r1["iterations"] == 8  # the cap rounded up to whole periods
    assert not r2["converged"] and r2["iterations"] == 4 and not x2.any()
    for M in Ms:
        M.close()


def test_stats_and_errors(cb):
    A = matgen.laplacian_2d(20)
    M = cb.CbMatrix.from_csr(A)
    R = cb.CbMatrix.from_csr(matgen.random_csr(30, 40, 0.2, 1))
    P = cb.CbMatrix.from_csr(A, lb_mode="paper")
    with cb.CbServer() as S:
        with pytest.raises(cb.CbError) as e:
            S.add_matrix(P)
        assert e.value.status == cb.CB_ERROR_NOT_SUPPORTED
        mid, rid = S.add_matrix(M), S.add_matrix(R)
        with pytest.raises(cb.CbError):
            S.submit_cg(rid, np.ones(40), np.zeros(40))  # not square
        with pytest.raises(ValueError):
            S.submit_cg(mid, np.ones(A.n, np.float32), np.zeros(A.n, np.float32))  # wrong vector type
        ts = [S.submit_cg(mid, matgen.vector(A.n, i), np.zeros(A.n)) for i in range(6)]
        for t in ts:
            assert S.wait(t)["converged"]
        with pytest.raises(cb.CbError):
            S.poll(10 ** 9)
        st = S.stats()
    assert st["cg_done"] == 6 and st["completed"] == 6 and st["submitted"] == 6
    assert 0 < st["p50_us"] <= st["p99_us"] and st["solves_per_s"] > 0 and st["steps"] > 0
    for h in (M, R, P):
        h.close()


def test_many_requests_submitted_while_the_worker_admits(cb):
    """Hundreds of submissions racing the worker's admission pass (the queue grows while the
    worker walks it)."""
    A, P = matgen.block_3d(4, seed=2), matgen.poisson_3d(7)
    MA, MP = cb.CbMatrix.from_csr(A), cb.CbMatrix.from_csr(P)
    rng = np.random.default_rng(9)
    with cb.CbServer(max_active=16) as S:
        a, p = S.add_matrix(MA), S.add_matrix(MP)
        jobs = []
        for j in range(400):
            if j % 5 == 0:
                b = matgen.vector(P.n, 200 + j)
                x = np.zeros(P.n)
                jobs.append(("cg", b, x, S.submit_cg(p, b, x, rtol=1e-9)))
            else:
                X = rng.uniform(-1, 1, A.n)
                Y = np.zeros(A.m)
                jobs.append(("spmm", X, Y, S.submit_spmm(a, X, Y)))
        for kind, u, v, t in jobs:
            r = S.wait(t)
            assert r["status"] == cb.CB_SUCCESS
            if kind == "cg":
                assert r["converged"] and solvers.residual(P, u, v) <= 2e-9
            else:
                e, viol, _ = oracle.scaled_error(v, oracle.spmv(A, u, comp=True), oracle.scale(A, u), 1e-12)
                assert viol == 0
        assert S.stats()["completed"] == 400
    MA.close()
    MP.close()


def run_refined(cb, specs, mix=False, **opts):
    """Refined solves (CB_REQ_CG_REFINE): specs of (A, low value type, seed of b); each request
    multiplies by the FP32/BF16 copy and replaces its residual with the FP64 matrix's.  With mix,
    plain FP64 and FP32 solves of the same matrices and SpMM requests run beside them.  Returns
    [(x, response)] of the refined requests in submission order."""
    mats, out = [], []
    with cb.CbServer(**opts) as S:
        tickets, extra = [], []
        for i, (A, low, seed) in enumerate(specs):
            Mh, Ml = cb.CbMatrix.from_csr(A), cb.CbMatrix.from_csr(A, value_type=low)
            mats += [Mh, Ml]
            h, lo = S.add_matrix(Mh), S.add_matrix(Ml)
            b = matgen.vector(A.n, seed)
            x = np.zeros(A.n)
            tickets.append((x, S.submit_cg_refine(h, lo, b, x, rtol=1e-10, max_iter=3000)))
            if mix:
                b2, x2 = matgen.vector(A.n, seed + 1), np.zeros(A.n)
                extra.append(S.submit_cg(h, b2, x2, rtol=1e-9))
                b3, x3 = matgen.vector(A.n, seed + 2).astype(np.float32), np.zeros(A.n, np.float32)
                extra.append(S.submit_cg(lo, b3, x3, rtol=1e-5))
                X, Y = np.random.default_rng(seed).uniform(-1, 1, (A.n, 3)), np.zeros((A.m, 3))
                extra.append(S.submit_spmm(h, X, Y))
        for x, t in tickets:
            out.append((x, S.wait(t)))
        for t in extra:
            assert S.wait(t)["status"] == cb.CB_SUCCESS
        stats = S.stats()
    for M in mats:
        M.close()
    return out, stats


def test_refined_solves_reach_the_true_residual_alone_and_in_a_mix(cb):
    """CB_REQ_CG_REFINE: FP32/BF16 products, FP64 residual replacement; every solve ends with a
    true residual <= 1e-10 (checked by the oracle on the FP64 matrix), and a solve's result is the
    same served alone and among other solves and SpMM requests."""
    spd = spd_matrices()
    # BF16 copies only of the operators whose values BF16 holds exactly (the scaled Poisson's are
    # rounded, and BF16 products then stall the replacement scheme)
    specs = [(A, low, 90 + 4 * i + j) for i, A in enumerate(spd) for j, low in enumerate(("f32", "bf16"))
             if low == "f32" or i < len(spd) - 1]
    alone = [run_refined(cb, [s])[0][0] for s in specs]
    mixed, stats = run_refined(cb, specs, mix=True, max_active=6)
    assert stats["active_peak"] > 1
    for (A, low, seed), (xa, ra), (xm, rm) in zip(specs, alone, mixed):
        b = matgen.vector(A.n, seed)
        for x, r in ((xa, ra), (xm, rm)):
            assert r["status"] == cb.CB_SUCCESS and r["converged"], (A.name, low, r)
            assert r["replacements"] >= 1 and r["rel_residual"] <= 1e-10
            assert solvers.residual(A, b, x) <= 1.5e-10, (A.name, low, solvers.residual(A, b, x))
        shared = cb.CbMatrix.from_csr(A, device=False, value_type=low).info["shared_panels"] + \
            cb.CbMatrix.from_csr(A, device=False).info["shared_panels"]
        if shared == 0:
            assert ra["iterations"] == rm["iterations"] and ra["replacements"] == rm["replacements"]
            assert np.array_equal(xa, xm), (A.name, low, np.abs(xa - xm).max())


def test_refined_solve_matches_cb_cg_refine_iterations(cb):
    """The served refined solve takes about the iterations of the one-matrix cb_cg_refine
    (CB_REFINE_REPLACE) on the same system: the same method, checked at the same period."""
    A = matgen.poisson_3d(14)
    b = matgen.vector(A.n, 5)
    [(x, r)], _ = run_refined(cb, [(A, "bf16", 5)], check_every=8)
    Mh, Ml = cb.CbMatrix.from_csr(A), cb.CbMatrix.from_csr(A, value_type="bf16")
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = Mh.cg_refine(Ml, torch.from_numpy(b).to("cuda"), xd, rtol=1e-10, max_iter=3000, check_every=8)
    Mh.close()
    Ml.close()
    assert res["converged"] and r["converged"]
    assert abs(res["iterations"] - r["iterations"]) <= 3 * 8, (res, r)
    assert solvers.residual(A, b, x) <= 1.5e-10


def test_refined_request_errors(cb):
    A = matgen.laplacian_2d(12)
    B = matgen.laplacian_2d(13)
    Mh, Ml, M32w, Mb = (cb.CbMatrix.from_csr(A), cb.CbMatrix.from_csr(A, value_type="bf16"),
                        cb.CbMatrix.from_csr(A, value_type="f32", vector_f64=1),
                        cb.CbMatrix.from_csr(B, value_type="f32"))
    with cb.CbServer() as S:
        h, lo, w, other = (S.add_matrix(M) for M in (Mh, Ml, M32w, Mb))
        b, x = np.ones(A.n), np.zeros(A.n)
        for hi, low in ((lo, lo), (h, h), (h, w), (h, other), (h, 99)):
            with pytest.raises(cb.CbError) as e:
                S.submit_cg_refine(hi, low, b, x)
            assert e.value.status == cb.CB_ERROR_INVALID_VALUE
        with pytest.raises(ValueError):
            S.submit_cg_refine(h, lo, b.astype(np.float32), x)  # b and x are double
        t = S.submit_cg_refine(h, lo, b, x)
        assert S.wait(t)["converged"]
    for M in (Mh, Ml, M32w, Mb):
        M.close()
