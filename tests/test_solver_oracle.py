"""Pins of the CG oracle against facts it does not compute itself (a direct
sparse solve, exact termination on a matrix with few distinct eigenvalues,
exact breakdown on an indefinite matrix, special cases), and the host-side
checks of the solver entry points (option defaults, argument errors), which
need no GPU."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle import solvers
from paper_2605_18515_amd import matgen


def scipy_of(A):
    return sp.csr_matrix((A.values, A.col_idx, A.row_ptr), shape=(A.m, A.n))


def diag(values):
    n = len(values)
    return matgen.Csr(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
                      np.asarray(values, np.float64))


@pytest.mark.parametrize("side", [8, 20])
def test_cg_matches_direct_solve(side):
    A = matgen.laplacian_2d(side)
    b = matgen.vector(A.n, 5)
    xs = spla.spsolve(scipy_of(A).tocsc(), b)
    x, it, conv, brk = solvers.cg(A, b, rtol=1e-12)
    assert conv and not brk and 0 < it <= A.n
    # |x - x*| <= cond(A) |r| / |b| |x*|; the 2D Dirichlet Laplacian has cond < (2 (side + 1) / pi)^2
    cond = (2 * (side + 1) / np.pi) ** 2
    assert np.linalg.norm(x - xs) <= 2 * cond * 1e-12 * np.linalg.norm(xs)
    assert solvers.residual(A, b, x) <= 1e-12


def test_cg_terminates_in_distinct_eigenvalue_steps():
    # in exact arithmetic CG ends after as many steps as A has distinct eigenvalues (here 4)
    vals = np.tile([1.0, 2.0, 4.0, 8.0], 50)
    A = diag(vals)
    b = matgen.vector(A.n, 2)
    x, it, conv, _ = solvers.cg(A, b, rtol=1e-13)
    assert conv and it <= 4
    np.testing.assert_allclose(x, b / vals, rtol=1e-12)


def test_cg_start_at_solution_and_zero_rhs():
    A = matgen.poisson_3d(6)
    xs = np.round(matgen.vector(A.n, 3) * 64) / 64
    b = oracle.spmv(A, xs)  # exact: small dyadic values
    x, it, conv, _ = solvers.cg(A, b, x0=xs)
    assert conv and it == 0 and np.array_equal(x, xs)
    x, it, conv, _ = solvers.cg(A, np.zeros(A.n))
    assert conv and it == 0 and not x.any()


def test_cg_breakdown_on_indefinite_matrix():
    # p = r = (1, 1), A p = (1, -1): (A p, p) = 0 exactly
    x, it, conv, brk = solvers.cg(diag([1.0, -1.0]), np.ones(2))
    assert brk and not conv and it == 1


def test_residual_special_cases():
    A = matgen.laplacian_2d(5)
    b = matgen.vector(A.n, 4)
    assert solvers.residual(A, b, np.zeros(A.n)) == pytest.approx(1.0, rel=1e-15)
    assert solvers.residual(A, np.zeros(A.n), np.zeros(A.n)) == 0.0
    # A = 2 I, b = (3, 4), x = 0: |r| / |b| = 1; x = (1, 1): r = (1, 2), |r| / |b| = sqrt(5) / 5
    assert solvers.residual(diag([2.0, 2.0]), np.array([3.0, 4.0]), np.ones(2)) == pytest.approx(5 ** 0.5 / 5,
                                                                                                   rel=1e-15)


# ---------------------------------------------------------------- host-side checks of the C ABI


@pytest.fixture(scope="module")
def cb():
    from paper_2605_18515_amd import cbspmv

    return cbspmv


def test_cg_options_default(cb):
    o = cb.cb_cg_options_default()
    assert o.struct_size == ctypes.sizeof(cb.CbCgOptions)
    assert (o.max_iter, o.rtol, o.check_every, o.max_refine, o.inner_rtol) == (10000, 1e-10, 16, 50, 1e-4)
    assert (o.refine_method, o.replace_factor) == (cb.CB_REFINE_REPLACE, 1e-2)
    assert ctypes.sizeof(cb.CbCgResult) == 40 and ctypes.sizeof(cb.CbCgOptions) == 64
    with pytest.raises(ValueError):
        cb.cb_cg_options_default(tolerance=1.0)


def test_cg_rejects_host_handles_and_bad_arguments(cb):
    A = matgen.laplacian_2d(4)
    h = cb.cb_create_host(A.m, A.n, A.nnz, A.row_ptr, A.col_idx, A.values)
    try:
        with pytest.raises(cb.CbError) as e:
            cb.cb_cg_workspace_bytes(h)
        assert e.value.status == cb.CB_ERROR_NOT_SUPPORTED
        with pytest.raises(cb.CbError) as e:
            cb.cb_cg(h, 0, 0, 0, 0)
        assert e.value.status == cb.CB_ERROR_NOT_SUPPORTED
        with pytest.raises(cb.CbError) as e:
            cb.cb_cg_refine(h, h, 0, 0, 0, 0)
        assert e.value.status == cb.CB_ERROR_NOT_SUPPORTED
        for bad in ({"max_iter": 0}, {"check_every": 0}, {"rtol": -1.0}, {"inner_rtol": 1.0}, {"max_refine": 0},
                    {"replace_factor": 0.0}, {"replace_factor": 1.0}, {"refine_method": 2}):
            with pytest.raises(cb.CbError) as e:
                cb.cb_cg(h, 0, 0, 0, 0, cb.cb_cg_options_default(**bad))
            assert e.value.status == cb.CB_ERROR_INVALID_VALUE
        o = cb.cb_cg_options_default()
        o.struct_size = 8
        with pytest.raises(cb.CbError) as e:
            cb.cb_cg(h, 0, 0, 0, 0, o)
        assert e.value.status == cb.CB_ERROR_INVALID_VALUE
    finally:
        cb.cb_destroy(h)
    for f in (lambda: cb.cb_cg_workspace_bytes(None), lambda: cb.cb_cg(None, 0, 0, 0, 0)):
        with pytest.raises(cb.CbError) as e:
            f()
        assert e.value.status == cb.CB_ERROR_INVALID_VALUE


# ---------------------------------------------------------------- serving loop, host side


def test_server_option_defaults_and_struct_sizes(cb):
    o = cb.cb_server_options_default()
    assert (o.max_active, o.arena_bytes, o.check_every, o.use_graph, o.spmm_streams) == (64, 1 << 30, 8, 1, 2)
    assert [ctypes.sizeof(t) for t in (cb.CbServerOptions, cb.CbRequest, cb.CbResponse, cb.CbServerStats)] == \
        [64, 96, 56, 144]
    with pytest.raises(ValueError):
        cb.cb_server_options_default(slots=3)


def test_server_rejects_bad_options_and_null_arguments(cb):
    lib = cb.library_handle()
    for bad in ({"max_active": 0}, {"check_every": 0}, {"use_graph": 2}, {"spmm_streams": 0}, {"arena_bytes": 16}):
        h = ctypes.c_void_p()
        st = lib.cb_server_create(ctypes.byref(cb.cb_server_options_default(**bad)), ctypes.byref(h))
        assert st == cb.CB_ERROR_INVALID_VALUE, bad
    o = cb.cb_server_options_default()
    o.struct_size = 4
    assert lib.cb_server_create(ctypes.byref(o), ctypes.byref(ctypes.c_void_p())) == cb.CB_ERROR_INVALID_VALUE
    r = cb.CbRequest()
    t = ctypes.c_int64()
    assert lib.cb_server_submit(None, ctypes.byref(r), ctypes.byref(t)) == cb.CB_ERROR_INVALID_VALUE
    assert lib.cb_server_poll(None, 1, ctypes.byref(cb.CbResponse())) == cb.CB_ERROR_INVALID_VALUE
    assert lib.cb_server_wait(None, 1, ctypes.byref(cb.CbResponse())) == cb.CB_ERROR_INVALID_VALUE
    assert lib.cb_server_stats(None, ctypes.byref(cb.CbServerStats())) == cb.CB_ERROR_INVALID_VALUE
    assert lib.cb_server_add_matrix(None, None, ctypes.byref(ctypes.c_int32())) == cb.CB_ERROR_INVALID_VALUE
    assert lib.cb_server_destroy(None) == cb.CB_SUCCESS


# ---------------------------------------------------------------- autotuner, host side


def test_tune_option_defaults_and_argument_errors(cb):
    o = cb.cb_tune_options_default()
    assert (o.reps, o.max_candidates) == (20, cb.CB_TUNE_MAX_CANDIDATES)
    assert ctypes.sizeof(cb.CbTuneCandidate) == ctypes.sizeof(cb.CbOptions) + 32
    A = matgen.laplacian_2d(8)
    lib = cb.library_handle()
    rp, ci, va = (np.ascontiguousarray(A.row_ptr), np.ascontiguousarray(A.col_idx), np.ascontiguousarray(A.values))
    best = cb.CbOptions()
    for bad in ({"reps": 0}, {"max_candidates": 0}, {"max_candidates": cb.CB_TUNE_MAX_CANDIDATES + 1},
                {"spmm_k": -1}, {"spmm_k": 4097}):
        st = lib.cb_tune(None, A.m, A.n, A.nnz, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, None,
                         ctypes.byref(cb.cb_tune_options_default(**bad)), ctypes.byref(best), None, None)
        assert st == cb.CB_ERROR_INVALID_VALUE, bad
    st = lib.cb_tune(None, A.m, A.n, A.nnz, rp.ctypes.data, ci.ctypes.data, va.ctypes.data,
                     ctypes.byref(cb.cb_options_default(lb_mode=cb.CB_LB_PAPER)), None, ctypes.byref(best), None, None)
    assert st == cb.CB_ERROR_NOT_SUPPORTED
    st = lib.cb_tune(None, A.m, A.n, A.nnz, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, None, None, None, None,
                     None)
    assert st == cb.CB_ERROR_INVALID_VALUE
