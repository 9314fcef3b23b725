"""Pins of the CPU oracle against facts that do not come from the oracle itself:
dense and scipy products, exact arithmetic, closed forms of stencil operators,
invariants (identity, permutation, row sums, linearity, alpha/beta special
cases), hand-worked rounding cases and an exact-fraction brute force."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2605_18515_amd import matgen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def dense_of(A):
    D = np.zeros((A.m, A.n))
    rows = A.rows()
    D[rows, A.col_idx] = A.values
    return D


@pytest.mark.parametrize("seed", range(6))
def test_spmv_matches_dense_product(seed):
    rng = np.random.default_rng(100 + seed)
    m, n = int(rng.integers(1, 45)), int(rng.integers(1, 45))
    A = matgen.random_csr(m, n, float(rng.uniform(0.05, 0.6)), seed)
    x = matgen.vector(n, seed)
    y0 = rng.uniform(-1, 1, m)
    alpha, beta = float(rng.uniform(-2, 2)), float(rng.uniform(-2, 2))
    ref = alpha * (dense_of(A) @ x) + beta * y0
    for comp in (False, True):
        y = oracle.spmv(A, x, alpha, beta, y0, comp=comp)
        np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)
    ys = alpha * (sp.csr_matrix((A.values, A.col_idx, A.row_ptr), shape=(m, n)) @ x) + beta * y0
    np.testing.assert_allclose(oracle.spmv(A, x, alpha, beta, y0), ys, rtol=1e-13, atol=1e-13)


def test_non_square_is_not_transposed():
    # a 3 x 5 matrix: a transposed operand cannot even take x of length 5
    D = np.array([[1.0, 0, 2, 0, 0], [0, 0, 0, 3, 0], [4, 0, 0, 0, 5]])
    A = matgen.from_dense(D)
    x = np.array([1.0, 10, 100, 1000, 10000])
    assert oracle.spmv(A, x).tolist() == [201.0, 3000.0, 50004.0]


@pytest.mark.parametrize("seed", range(4))
def test_exact_dyadic_is_bitwise(seed):
    """p/64 values times q/64 inputs: every partial sum is exact in FP64, so
    any summation order must give the same bits as the dense product."""
    A = matgen.random_csr(60, 50, 0.3, seed, values="dyadic")
    x = matgen.vector(50, seed, dyadic=True)
    ref = dense_of(A) @ x
    y = oracle.spmv(A, x)
    assert np.array_equal(y.view(np.uint64), ref.view(np.uint64))


def test_compensated_matches_fsum():
    A = matgen.random_csr(30, 200, 0.8, 7)
    x = matgen.vector(200, 7) * np.geomspace(1e-8, 1e8, 200)
    yc = oracle.spmv(A, x, comp=True)
    rows = A.rows()
    for i in range(A.m):
        sel = rows == i
        exact = math.fsum((A.values[sel] * x[A.col_idx[sel]]).tolist())
        # products are rounded once each; the compensated sum of them is within
        # one unit of the correctly rounded sum of those same products
        assert abs(yc[i] - exact) <= 2 * np.spacing(abs(exact)) + 1e-300


def test_scale_is_abs_product():
    A = matgen.random_csr(25, 33, 0.4, 3)
    x = matgen.vector(33, 3)
    y0 = np.linspace(-2, 2, 25)
    s = oracle.scale(A, x, alpha=-1.5, beta=0.25, y0=y0)
    np.testing.assert_allclose(s, 1.5 * (np.abs(dense_of(A)) @ np.abs(x)) + 0.25 * np.abs(y0), rtol=1e-14)
    s0 = oracle.scale(A, x, alpha=2.0, beta=0.0, y0=np.full(25, np.nan))
    assert np.isfinite(s0).all()


def test_row_sums_identity_permutation():
    A = matgen.random_csr(40, 40, 0.2, 11)
    ones = np.ones(40)
    rs = np.zeros(40)
    np.add.at(rs, A.rows(), A.values)
    np.testing.assert_allclose(oracle.spmv(A, ones), rs, rtol=1e-14, atol=1e-15)
    x = matgen.vector(97, 1)
    I = matgen.identity(97)
    assert np.array_equal(oracle.spmv(I, x).view(np.uint64), x.view(np.uint64))
    P, pi = matgen.permutation(97, 5)
    assert np.array_equal(oracle.spmv(P, x).view(np.uint64), x[pi].view(np.uint64))


def test_linearity():
    A = matgen.random_csr(50, 64, 0.25, 4)
    x, z = matgen.vector(64, 1), matgen.vector(64, 2)
    a, b = 0.75, -1.25
    lhs = oracle.spmv(A, a * x + b * z)
    rhs = a * oracle.spmv(A, x) + b * oracle.spmv(A, z)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-13)


def test_alpha_beta_special_cases():
    A = matgen.random_csr(20, 20, 0.3, 9)
    x = matgen.vector(20, 9)
    y0 = matgen.vector(20, 10)
    assert np.array_equal(oracle.spmv(A, x, alpha=0.0, beta=0.5, y0=y0), 0.5 * y0)
    y = oracle.spmv(A, x, alpha=1.0, beta=0.0, y0=np.full(20, np.nan))
    assert np.isfinite(y).all()
    np.testing.assert_array_equal(oracle.spmv(A, x, 1.0, 1.0, y0) - y0, oracle.spmv(A, x, 1.0, 1.0, y0) - y0)
    np.testing.assert_allclose(oracle.spmv(A, x, 2.0, 1.0, y0), 2.0 * (dense_of(A) @ x) + y0, rtol=1e-14)


def test_laplacian_closed_forms():
    side = 12
    A = matgen.laplacian_2d(side)
    r = np.arange(side * side)
    i, j = r % side, r // side
    boundary_sides = (i == 0).astype(int) + (i == side - 1) + (j == 0) + (j == side - 1)
    # (A 1)_i = 4 - (number of neighbours) = number of missing neighbours
    assert np.array_equal(oracle.spmv(A, np.ones(side * side)), boundary_sides.astype(float))
    # a linear field is harmonic: interior rows of A (i + j) are exactly zero
    y = oracle.spmv(A, (i + j).astype(float))
    interior = (boundary_sides == 0)
    assert np.all(y[interior] == 0.0)


def test_poisson_closed_form():
    side = 7
    A = matgen.poisson_3d(side)
    r = np.arange(side ** 3)
    i, j, k = r % side, (r // side) % side, r // side ** 2
    missing = sum((c == 0).astype(int) + (c == side - 1) for c in (i, j, k))
    assert np.array_equal(oracle.spmv(A, np.ones(side ** 3)), missing.astype(float))


@pytest.mark.parametrize("k", [1, 3, 8])
def test_spmm_matches_dense(k):
    A = matgen.random_csr(33, 29, 0.3, k)
    X = matgen.rhs(29, k, k)
    Y0 = matgen.rhs(33, k, k + 100)
    ref = 0.5 * (dense_of(A) @ X) - 2.0 * Y0
    for comp in (False, True):
        np.testing.assert_allclose(oracle.spmm(A, X, 0.5, -2.0, Y0, comp=comp), ref, rtol=1e-13, atol=1e-13)
    # column j of the k-vector product equals the single-vector product
    for jj in range(k):
        np.testing.assert_array_equal(oracle.spmm(A, X)[:, jj], oracle.spmv(A, X[:, jj]))


def _parse(s):
    return float.fromhex(s) if "0x" in s else float(s)


def test_rounding_golden_cases():
    cases = json.load(open(os.path.join(GOLD, "rounding_cases.json")))["cases"]
    for s, b16, f32, why in cases:
        v = _parse(s)
        assert int(oracle.round_bf16_bits(v)[0]) == int(b16, 16), (s, why)
        assert int(oracle.round_f32_bits(v)[0]) == int(f32, 16), (s, why)


def test_f32_rounding_matches_hardware_conversion():
    rng = np.random.default_rng(1)
    v = np.concatenate([
        rng.standard_normal(20000) * np.exp2(rng.integers(-160, 140, 20000)),
        np.array([0.0, -0.0, np.inf, -np.inf, 3.5e38, -3.5e38, 1e-46, 7e-46, 1.4e-45]),
    ])
    with np.errstate(over="ignore"):
        ref = v.astype(np.float32).view(np.uint32)
    assert np.array_equal(oracle.round_f32_bits(v), ref)


def _bf16_brute(v: float) -> int:
    """Nearest bf16 by exact rational comparison of the two neighbouring
    candidates (enumerated from bit patterns), ties to the even pattern."""
    if math.isnan(v):
        raise ValueError
    sign = 0x8000 if math.copysign(1.0, v) < 0 else 0
    a = abs(v)
    if math.isinf(a):
        return sign | 0x7F80

    def value(bits):  # non-negative bf16 pattern -> Fraction (bits < 0x7F80)
        e, mnt = bits >> 7, bits & 0x7F
        if e == 0:
            return Fraction(mnt, 1 << 7) * Fraction(2) ** -126
        return (1 + Fraction(mnt, 1 << 7)) * Fraction(2) ** (e - 127)

    fa = Fraction(a)
    lo, hi = 0, 0x7F80
    while hi - lo > 1:  # largest pattern with value <= a
        mid = (lo + hi) // 2
        if value(mid) <= fa:
            lo = mid
        else:
            hi = mid
    below = lo
    above = below + 1
    vb = value(below)
    if vb == fa:
        return sign | below
    va = value(above) if above < 0x7F80 else (1 + Fraction(1)) * Fraction(2) ** 127  # 2^128 stands in for Inf
    db, da = fa - vb, va - fa
    pick = below if (db < da or (db == da and below % 2 == 0)) else above
    return sign | pick


def test_bf16_rounding_matches_exact_brute_force():
    rng = np.random.default_rng(2)
    v = np.concatenate([
        rng.standard_normal(3000) * np.exp2(rng.integers(-140, 128, 3000)),
        # values sitting exactly on or next to bf16 ties
        (1 + (2 * rng.integers(0, 128, 500) + 1) / 256.0) * np.exp2(rng.integers(-20, 20, 500)),
        np.nextafter((1 + (2 * rng.integers(0, 128, 200) + 1) / 256.0), 2.0),
        np.nextafter((1 + (2 * rng.integers(0, 128, 200) + 1) / 256.0), 0.0),
    ])
    got = oracle.round_bf16_bits(v)
    for vi, g in zip(v.tolist(), got.tolist()):
        assert g == _bf16_brute(vi), (vi.hex(), hex(g))


def test_nan_stays_quiet_nan():
    nan_payload = np.frombuffer(np.uint64(0x7FF0000000000001).tobytes(), dtype=np.float64)[0]  # signalling
    b = int(oracle.round_bf16_bits(nan_payload)[0])
    f = int(oracle.round_f32_bits(nan_payload)[0])
    assert (b & 0x7F80) == 0x7F80 and (b & 0x40)
    assert (f & 0x7F800000) == 0x7F800000 and (f & 0x400000)


def test_scaled_error_rules():
    yref = np.array([1.0, 2.0, 0.0, np.nan, np.inf, 5.0])
    scl = np.array([1.0, 1.0, 0.0, 1.0, 1.0, 1.0])
    e, v, _ = oracle.scaled_error(yref.copy(), yref, scl, 1e-12)
    assert e == 0.0 and v == 0
    y = yref.copy(); y[0] += 1e-13
    e, v, w = oracle.scaled_error(y, yref, scl, 1e-12)
    assert v == 0 and 0 < e < 1e-12
    y = yref.copy(); y[1] += 1e-11
    assert oracle.scaled_error(y, yref, scl, 1e-12)[1] == 1
    y = yref.copy(); y[2] = 1e-300  # zero scale demands an exact match
    assert oracle.scaled_error(y, yref, scl, 1e-12)[1] == 1
    y = yref.copy(); y[3] = 0.0     # NaN reference demands NaN
    assert oracle.scaled_error(y, yref, scl, 1e-12)[1] == 1
    y = yref.copy(); y[4] = -np.inf  # infinite reference demands the same infinity
    assert oracle.scaled_error(y, yref, scl, 1e-12)[1] == 1
    y = yref.copy(); y[5] = np.nan
    assert oracle.scaled_error(y, yref, scl, 1e-12)[1] == 1


def test_compensated_sum_with_non_finite_terms():
    """An Inf or NaN product makes the row the plain IEEE sum: +Inf stays +Inf,
    Inf - Inf and NaN give NaN, whatever the summation variant."""
    D = np.array([[1.0, np.inf, 2.0, 0.0],
                  [1.0, np.inf, -np.inf, 0.0],
                  [np.nan, 1.0, 0.0, 0.0],
                  [1e308, 1e308, 0.0, 0.0],
                  [3.0, -1.0, 0.0, 1.0]])
    keep = np.ones_like(D, dtype=bool)
    A = matgen.from_dense(D, keep_zeros_mask=keep)
    x = np.array([1.0, 2.0, 3.0, 4.0])
    with np.errstate(invalid="ignore", over="ignore"):
        ref = D @ x
    for comp in (False, True):
        y = oracle.spmv(A, x, comp=comp)
        assert np.array_equal(np.isnan(y), np.isnan(ref))
        assert np.array_equal(y[~np.isnan(y)], ref[~np.isnan(ref)])
        Y = oracle.spmm(A, np.stack([x, 2 * x], axis=1), comp=comp)
        assert np.array_equal(np.isnan(Y[:, 0]), np.isnan(ref)) and Y[0, 0] == np.inf and Y[3, 1] == np.inf


@pytest.mark.parametrize("threads", [1, 4])
def test_parallel_csr_product_equals_the_plain_loop(threads):
    # each row summed in entry order either way: bit for bit
    A = matgen.power_law(3000, seed=4, max_len=500, window=100)
    x = matgen.vector(A.n, 2)
    y = np.empty(A.m)
    rp, ci, va = (np.ascontiguousarray(A.row_ptr), np.ascontiguousarray(A.col_idx),
                  np.ascontiguousarray(A.values))
    oracle.lib().oracle_spmv_csr_par(A.m, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, x.ctypes.data, 1.5,
                                     y.ctypes.data, threads)
    assert np.array_equal(y, oracle.spmv(A, x, alpha=1.5))
