"""GPU tests of the autotuner (cb_tune): the tuned handle and every candidate it timed compute
the product within the storage precision's tolerance of the oracle, the chosen candidate is
the fastest up to the 1 % keep rule, and the storage and vector types asked for are kept."""
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


def check(cb, M, A, vt, wide=False):
    x = matgen.vector(A.n, 3)
    dt = torch.float64 if vt == "f64" or wide else torch.float32
    y = torch.full((A.m,), float("nan"), dtype=dt, device="cuda")
    M.spmv(torch.from_numpy(x).to("cuda", dt), y)
    torch.cuda.synchronize()
    e, viol, _ = oracle.scaled_error(y.cpu().double().numpy(), oracle.spmv(A, x, comp=True), oracle.scale(A, x),
                                     TOL[vt])
    assert viol == 0, (vt, e)


@pytest.mark.parametrize("name,vt,wide", [("block", "f64", 0), ("power", "f32", 0), ("poisson", "bf16", 1),
                                          ("lap", "f64", 0)])
def test_tuned_handle_and_every_candidate_are_correct(cb, name, vt, wide):
    A = {"block": lambda: matgen.block_3d(14, seed=1), "power": lambda: matgen.power_law(30000, seed=2, max_len=3000),
         "poisson": lambda: matgen.poisson_3d(24), "lap": lambda: matgen.laplacian_2d(64)}[name]()
    M, best, cands = cb.cb_tune(A, value_type=vt, vector_f64=wide, reps=5)
    print(f"[tune {name} {vt}] " + "; ".join(
        f"S={c['tile_dim']} k{c['spmv_kernel']} agg={c['col_agg']} th=({c['opt']['th1']},{c['opt']['th2']}) "
        f"rr={c['row_reduce']} lb={c['opt']['lb_mode']} wn={c['opt']['wave_nnz']} {c['us']:.1f}us"
        f"{' *' if c['best'] else ''}" for c in cands))
    assert 5 <= len(cands) <= cb.CB_TUNE_MAX_CANDIDATES and sum(c["best"] for c in cands) == 1
    b = next(c for c in cands if c["best"])
    assert b["opt"] == best and b["us"] <= min(c["us"] for c in cands) / 0.99 + 1e-9
    assert best["value_type"] == cb.VALUE_TYPES[vt] and best["vector_f64"] == wide
    # both sub-block sizes and both natural-order kernels were timed
    assert {c["tile_dim"] for c in cands} == {8, 16} and {c["spmv_kernel"] for c in cands} == {0, 2}
    check(cb, M, A, vt, wide)
    assert M.info["col_agg"] == b["col_agg"] and M.info["row_reduce"] == b["row_reduce"]
    assert M.info["tile_dim"] == b["tile_dim"] and M.info["spmv_kernel"] == b["spmv_kernel"]
    M.close()
    for c in cands:
        Mc = cb.CbMatrix.from_csr(A, **c["opt"])
        check(cb, Mc, A, vt, wide)
        Mc.close()


def test_tuner_without_keeping_the_handle(cb):
    A = matgen.laplacian_2d(40)
    M, best, cands = cb.cb_tune(A, keep=False, reps=3)
    assert M is None and len(cands) >= 5 and best["lb_mode"] in (cb.CB_LB_CONTIGUOUS, cb.CB_LB_NONE)
    assert {c["opt"]["lb_mode"] for c in cands} == {cb.CB_LB_CONTIGUOUS, cb.CB_LB_NONE}


@pytest.mark.parametrize("k", [8, 32])
def test_tuner_for_k_right_hand_sides(cb, k):
    """spmm_k: the candidates are timed on cb_spmm with k columns; the tuned handle's SpMM meets the
    oracle."""
    A = matgen.block_3d(12, seed=4)
    M, best, cands = cb.cb_tune(A, reps=3, spmm_k=k)
    assert len(cands) >= 5 and {c["tile_dim"] for c in cands} == {8, 16}
    X = matgen.rhs(A.n, k, 5)
    Yd = torch.full((A.m, k), float("nan"), dtype=torch.float64, device="cuda")
    M.spmm(torch.from_numpy(X).cuda(), Yd)
    torch.cuda.synchronize()
    e, viol, _ = oracle.scaled_error(Yd.cpu().numpy(), oracle.spmm(A, X, comp=True), oracle.spmm_scale(A, X), 1e-12)
    assert viol == 0, e
    M.close()
