"""CPU oracle for the solvers built on the sparse product -- TEST INFRASTRUCTURE ONLY.

Conjugate gradient and the true residual that the solver tests are checked against.
These are not part of the paper's method: they consume its product (y = A x,
Section 2.1) as the adjacent step of a mixed-precision solver.  CG is the
method of Hestenes and Stiefel (1952), as stated in Saad, "Iterative Methods
for Sparse Linear Systems" (2nd ed.), Algorithm 6.18, in FP64 with the oracle's
plain product.  Only ``tests/`` may import this module.
"""
from __future__ import annotations

import math

import numpy as np

from . import spmv


def residual(A, b, x) -> float:
    """|b - A x| / |b| in FP64 (|b - A x| when b = 0), the product Neumaier-compensated."""
    b = np.asarray(b, np.float64)
    x = np.asarray(x, np.float64)
    r = spmv(A, x, alpha=-1.0, beta=1.0, y0=b, comp=True)
    nb = math.sqrt(float(np.dot(b, b)))
    nr = math.sqrt(float(np.dot(r, r)))
    return nr / nb if nb > 0 else nr


def cg(A, b, x0=None, rtol=1e-10, max_iter=10000):
    """Plain FP64 CG from x0 (zeros when None) until |r_j| <= rtol |b| on the recurrence residual.

    Steps per iteration: alpha = (r, r) / (A p, p); x += alpha p; r -= alpha A p;
    beta = (r_new, r_new) / (r, r); p = r_new + beta p.  Returns (x, iterations, converged,
    breakdown), breakdown True when (A p, p) <= 0 (A not positive definite along p)."""
    b = np.asarray(b, np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, np.float64)
    r = b - spmv(A, x)
    p = r.copy()
    rr = float(np.dot(r, r))
    target = rtol * math.sqrt(float(np.dot(b, b)))
    if math.sqrt(rr) <= target:
        return x, 0, True, False
    for j in range(1, max_iter + 1):
        q = spmv(A, p)
        pq = float(np.dot(p, q))
        if not (pq > 0.0 and math.isfinite(pq)):
            return x, j, False, True
        alpha = rr / pq
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(np.dot(r, r))
        if math.sqrt(rr_new) <= target:
            return x, j, True, False
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, max_iter, False, False
