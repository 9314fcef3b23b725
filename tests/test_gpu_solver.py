"""GPU tests of the solvers built on the CB product: FP64 CG, CG on FP32
storage, and FP64 iterative refinement around a CG on an FP32 or BF16 copy of
the matrix.  Checked by the oracle: the FP64 true residual |b - A x| / |b| of the
returned x, agreement with the oracle's FP64 CG within the bound the condition
number gives, exact breakdown on a negative definite matrix, and the argument
errors of the entry points."""
import math

import numpy as np
import pytest

from oracle import solvers
from paper_2605_18515_amd import matgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2605_18515_amd import cbspmv

    torch.cuda.init()
    return cbspmv


def poisson_cond(side):
    """Condition number of the 3D Dirichlet 7-point operator on side^3 nodes (closed form)."""
    h = math.pi / (side + 1)
    return (6 + 6 * math.cos(h)) / (6 - 6 * math.cos(h))


def scaled_poisson(side, seed=3):
    """S A S with the 3D Poisson operator A and S = diag(s), s uniform in [0.8, 1.25]: SPD, with
    values that FP32 and BF16 do not hold exactly, condition number at most (1.25 / 0.8)^2 cond(A)."""
    A = matgen.poisson_3d(side)
    s = np.random.default_rng(seed).uniform(0.8, 1.25, A.n)
    return matgen.Csr(A.m, A.n, A.row_ptr, A.col_idx, s[A.rows()] * A.values * s[A.col_idx])


def dev(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)


def host(t):
    return t.cpu().double().numpy()


@pytest.mark.parametrize("x0_seed", [None, 9])
def test_cg_f64_matches_oracle(cb, x0_seed):
    side = 24
    A = matgen.poisson_3d(side)
    b = matgen.vector(A.n, 5)
    x0 = np.zeros(A.n) if x0_seed is None else matgen.vector(A.n, x0_seed)
    M = cb.CbMatrix.from_csr(A, value_type="f64")
    xd = dev(x0)
    res = M.cg(dev(b), xd, rtol=5e-11)
    torch.cuda.synchronize()
    M.close()
    x = host(xd)
    xo, ito, conv_o, _ = solvers.cg(A, b, x0=x0, rtol=5e-11)
    true = solvers.residual(A, b, x)
    print(f"[cg f64 poisson {side}^3 x0={x0_seed}] iters {res['iterations']} (oracle {ito}), "
          f"true residual {true:.3e} (reported {res['rel_residual']:.3e})")
    assert res["converged"] and conv_o
    assert true <= 1e-10
    assert abs(res["rel_residual"] - true) <= 1e-3 * true + 1e-15
    # both stop when the residual is within 5e-11 |b|; |x - x*| <= cond * |r| / |b| * |x*| for each
    assert np.linalg.norm(x - xo) <= 2 * poisson_cond(side) * 1e-10 * np.linalg.norm(xo)
    # the device checks convergence every check_every (16) iterations
    assert ito - 2 <= res["iterations"] <= ito + 16 + 2


def test_cg_f32_storage(cb):
    A = matgen.poisson_3d(20)
    b = matgen.vector(A.n, 6)
    M = cb.CbMatrix.from_csr(A, value_type="f32")
    xd = torch.zeros(A.n, dtype=torch.float32, device="cuda")
    res = M.cg(dev(b, torch.float32), xd, rtol=1e-5, check_every=4)
    torch.cuda.synchronize()
    M.close()
    # the stored values (6, -1) and b rounded to FP32 define the solved system; check in FP64
    bf = b.astype(np.float32).astype(np.float64)
    true = solvers.residual(A, bf, host(xd))
    print(f"[cg f32 poisson 20^3] iters {res['iterations']} recurrence {res['rel_residual']:.3e} true {true:.3e}")
    assert res["converged"] and res["rel_residual"] <= 1e-5
    assert true <= 1e-4


@pytest.mark.parametrize("method", ["replace", "restart"])
@pytest.mark.parametrize("low", ["f32", "bf16", "f32-wide", "bf16-wide"])
def test_cg_refine_reaches_fp64_accuracy(cb, low, method):
    side = 24
    A = scaled_poisson(side)
    b = matgen.vector(A.n, 7)
    M = cb.CbMatrix.from_csr(A, value_type="f64")
    L = cb.CbMatrix.from_csr(A, value_type=low.split("-")[0], vector_f64=int(low.endswith("wide")))
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    meth = cb.CB_REFINE_REPLACE if method == "replace" else cb.CB_REFINE_RESTART
    res = M.cg_refine(L, dev(b), xd, rtol=5e-11, refine_method=meth)
    x64 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res64 = M.cg(dev(b), x64, rtol=5e-11)
    torch.cuda.synchronize()
    M.close()
    L.close()
    x = host(xd)
    true = solvers.residual(A, b, x)
    print(f"[cg refine {low} {method}] refinements {res['refinements']} iterations {res['iterations']} "
          f"true residual {true:.3e}; fp64 cg iters {res64['iterations']}")
    assert res["converged"] and res["refinements"] >= (1 if method == "replace" else 2)
    assert true <= 1e-10
    assert abs(res["rel_residual"] - true) <= 1e-3 * true + 1e-15
    xo = host(x64)
    assert res64["converged"] and solvers.residual(A, b, xo) <= 1e-10
    cond = (1.25 / 0.8) ** 2 * poisson_cond(side)
    assert np.linalg.norm(x - xo) <= 2 * cond * 1e-10 * np.linalg.norm(xo)
    xr, _, conv_o, _ = solvers.cg(A, b, rtol=5e-11)
    assert conv_o and np.linalg.norm(x - xr) <= 2 * cond * 1e-10 * np.linalg.norm(xr)


def test_cg_breakdown_on_negative_definite(cb):
    A = matgen.laplacian_2d(12)
    A = matgen.Csr(A.m, A.n, A.row_ptr, A.col_idx, -A.values)
    b = matgen.vector(A.n, 8)
    _, ito, conv_o, brk = solvers.cg(A, b)
    assert brk and not conv_o and ito == 1
    M = cb.CbMatrix.from_csr(A, value_type="f64")
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = M.cg(dev(b), xd, check_every=1)
    torch.cuda.synchronize()
    M.close()
    assert not res["converged"] and res["iterations"] == 1
    # the failed step left x at its start
    assert not host(xd).any()


def test_cg_zero_rhs_and_empty(cb):
    A = matgen.laplacian_2d(6)
    M = cb.CbMatrix.from_csr(A, value_type="f64")
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = M.cg(torch.zeros(A.n, dtype=torch.float64, device="cuda"), xd)
    torch.cuda.synchronize()
    M.close()
    assert res["converged"] and res["iterations"] == 0 and not host(xd).any()
    E = matgen.Csr(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    M = cb.CbMatrix.from_csr(E, value_type="f64")
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    res = M.cg(e, e)
    M.close()
    assert res["converged"] and res["iterations"] == 0


def test_cg_argument_errors(cb):
    A = matgen.laplacian_2d(6)
    M = cb.CbMatrix.from_csr(A, value_type="f64")
    L = cb.CbMatrix.from_csr(A, value_type="f32")
    R = cb.CbMatrix.from_csr(matgen.random_csr(36, 20, 0.2, 1), value_type="f64")
    b = torch.ones(A.n, dtype=torch.float64, device="cuda")
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    need = cb.cb_cg_workspace_bytes(M.handle)
    w = torch.empty(need, dtype=torch.uint8, device="cuda")
    try:
        with pytest.raises(cb.CbError) as e:
            cb.cb_cg(M.handle, b, x, w, need - 1)
        assert e.value.status == cb.CB_ERROR_INVALID_VALUE
        with pytest.raises(cb.CbError) as e:  # precisions swapped
            cb.cb_cg_refine(L.handle, M.handle, b, x, w, need)
        assert e.value.status == cb.CB_ERROR_INVALID_VALUE
        with pytest.raises(cb.CbError) as e:  # not square
            cb.cb_cg_workspace_bytes(R.handle)
        assert e.value.status == cb.CB_ERROR_INVALID_VALUE
        assert cb.cb_cg_workspace_bytes(M.handle, L.handle) > need
        res = cb.cb_cg(M.handle, b, x, w, need)
        torch.cuda.synchronize()
        assert res["converged"] and solvers.residual(A, np.ones(A.n), host(x)) <= 2e-10
    finally:
        for h in (M, L, R):
            h.close()
