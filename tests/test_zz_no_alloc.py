"""cb_cg_noalloc (CG with the library's fixed device workspace) against cb_cg with a caller
workspace, through the C ABI: two calls in a row, the second on a smaller matrix, each equal to the
existing entry point's solve within the bound the condition number gives (the arithmetic is the
same, so they normally agree bit for bit), each true FP64 residual checked by the oracle; a float
vector solve; and the refusal of a solve whose workspace exceeds the fixed size."""
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
    h = math.pi / (side + 1)
    return (6 + 6 * math.cos(h)) / (6 - 6 * math.cos(h))


def solve_both(cb, A, vtype, rtol, seed):
    dt = torch.float64 if vtype == "f64" else torch.float32
    b = matgen.vector(A.n, seed)
    M = cb.CbMatrix.from_csr(A, value_type=vtype)
    opt = cb.cb_cg_options_default(rtol=rtol, max_iter=4000)
    bd = torch.from_numpy(b).to("cuda", dt)
    # the existing entry point, with a workspace of its own
    x_ref = torch.zeros(A.n, dtype=dt, device="cuda")
    need = cb.cb_cg_workspace_bytes(M.handle)
    assert need <= cb.CB_CG_NOALLOC_MAX_BYTES
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    r_ref = cb.cb_cg(M.handle, bd, x_ref, work, need, opt)
    torch.cuda.synchronize()
    # the same solve on the library's fixed workspace
    x_na = torch.zeros(A.n, dtype=dt, device="cuda")
    r_na = cb.cb_cg_noalloc(M.handle, bd, x_na, opt)
    torch.cuda.synchronize()
    M.close()
    return b, x_ref.cpu().double().numpy(), r_ref, x_na.cpu().double().numpy(), r_na


def test_noalloc_cg_twice_second_smaller(cb):
    rtol = 1e-10
    for side in (60, 30):
        A = matgen.poisson_3d(side)
        print(f"[noalloc] FP64 Poisson {side}^3, n = {A.n}", flush=True)
        b, x_ref, r_ref, x_na, r_na = solve_both(cb, A, "f64", rtol, 5)
        assert r_ref["converged"] and r_na["converged"]
        assert r_na["iterations"] == r_ref["iterations"]
        for x in (x_ref, x_na):
            assert solvers.residual(A, b, x) <= rtol
        # two solutions with residuals <= rtol |b| differ by at most 2 rtol cond(A) relative
        d = np.linalg.norm(x_na - x_ref) / np.linalg.norm(x_ref)
        print(f"[noalloc] iterations {r_na['iterations']}, relative difference {d:.3e}, "
              f"bitwise equal {np.array_equal(x_na, x_ref)}", flush=True)
        assert d <= 2 * rtol * poisson_cond(side)


def test_noalloc_cg_float_vectors(cb):
    A = matgen.poisson_3d(24)
    b, x_ref, r_ref, x_na, r_na = solve_both(cb, A, "f32", 1e-5, 6)
    assert r_ref["converged"] and r_na["converged"]
    assert r_na["iterations"] == r_ref["iterations"]
    d = np.linalg.norm(x_na - x_ref) / np.linalg.norm(x_ref)
    assert d <= 2 * 1e-5 * poisson_cond(24)


def test_noalloc_refuses_a_solve_larger_than_its_workspace(cb):
    A = matgen.poisson_3d(143)  # n = 2,924,207: 24 n bytes of FP64 vectors exceed the 64 MiB array
    M = cb.CbMatrix.from_csr(A)
    need = cb.cb_cg_workspace_bytes(M.handle)
    assert need > cb.CB_CG_NOALLOC_MAX_BYTES
    bd = torch.ones(A.n, dtype=torch.float64, device="cuda")
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(cb.CbError) as ei:
        cb.cb_cg_noalloc(M.handle, bd, xd)
    assert ei.value.status == cb.CB_ERROR_INVALID_VALUE and "workspace" in str(ei.value)
    torch.cuda.synchronize()
    assert float(xd.abs().max()) == 0.0  # nothing ran
    M.close()
