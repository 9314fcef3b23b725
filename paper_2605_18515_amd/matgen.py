"""Seeded synthetic sparse matrices and dense operands.

These generators produce the workloads the library is measured and tested on:
matrices with the shapes, value distributions and structure of the paper's
evaluation families (stencils, block-structured FEM-like operators and
power-law graphs, Section 4), built from a seed instead of the SuiteSparse
files the paper used (not available here).  They hold none of the CB-SpMV
arithmetic: they only emit canonical CSR (int64 row pointers, int32 sorted
unique column indices, float64 values) and dense vectors, and are shared by the
tests, the benchmark and the oracle-driven checks.

Every random draw comes from ``numpy.random.default_rng`` (PCG64) seeded with
``[seed, stream]`` so the matrix, the input vector and each right-hand side have
independent, reproducible streams.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

STREAM_MATRIX = 0
STREAM_X = 1
STREAM_RHS = 2
STREAM_Y0 = 3


@dataclass
class Csr:
    m: int
    n: int
    row_ptr: np.ndarray  # int64[m+1]
    col_idx: np.ndarray  # int32[nnz]
    values: np.ndarray   # float64[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def rows(self) -> np.ndarray:
        """Row index of every stored entry (COO expansion of row_ptr)."""
        return np.repeat(np.arange(self.m, dtype=np.int32), np.diff(self.row_ptr))


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


def _from_slots(nrows: int, cols: np.ndarray, valid: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """cols/valid are (nrows, slots) with slots already in ascending column order."""
    counts = valid.sum(axis=1).astype(np.int64)
    row_ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, cols[valid].astype(np.int32)


def laplacian_2d(side: int) -> Csr:
    """2D 5-point Laplacian on a side x side grid, row = i + side*j, Dirichlet
    (no wrap): 4 on the diagonal, -1 to each existing neighbour."""
    N = side * side
    r = np.arange(N, dtype=np.int64)
    i, j = r % side, r // side
    offs = np.array([-side, -1, 0, 1, side], dtype=np.int64)
    cols = r[:, None] + offs[None, :]
    valid = np.stack([j > 0, i > 0, np.ones(N, bool), i < side - 1, j < side - 1], axis=1)
    row_ptr, col = _from_slots(N, cols, valid)
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    val = np.where(col == rows, 4.0, -1.0)
    return Csr(N, N, row_ptr, col, val, f"laplacian2d_{side}")


def poisson_3d(side: int) -> Csr:
    """3D 7-point Poisson operator on a side^3 grid, node = i + side*j + side^2*k,
    Dirichlet: 6 on the diagonal, -1 to each existing face neighbour (SPD)."""
    N = side ** 3
    s2 = side * side
    r = np.arange(N, dtype=np.int64)
    i, j, k = r % side, (r // side) % side, r // s2
    offs = np.array([-s2, -side, -1, 0, 1, side, s2], dtype=np.int64)
    valid = np.stack([k > 0, j > 0, i > 0, np.ones(N, bool), i < side - 1, j < side - 1, k < side - 1], axis=1)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(valid.sum(axis=1), out=row_ptr[1:])
    col = (r[:, None] + offs[None, :])[valid].astype(np.int32)
    del valid
    val = np.full(col.shape[0], -1.0)
    diag_pos = row_ptr[:-1] + (k > 0) + (j > 0) + (i > 0)
    val[diag_pos] = 6.0
    return Csr(N, N, row_ptr, col, val, f"poisson3d_{side}")


def block_3d(side: int = 100, dof: int = 3, shift: float = 10.0, seed: int = 1) -> Csr:
    """3D 7-point adjacency (self + 6 face neighbours, no wrap) on side^3 nodes,
    node = i + side*j + side^2*k, with ``dof`` unknowns per node (row = dof*node + d).
    Every (node, neighbour) pair is a dense dof x dof block of U[-1, 1] values;
    ``shift`` is added to each scalar diagonal entry (diagonal dominance)."""
    N = side ** 3
    s2 = side * side
    node = np.arange(N, dtype=np.int64)
    i, j, k = node % side, (node // side) % side, node // s2
    offs = np.array([-s2, -side, -1, 0, 1, side, s2], dtype=np.int64)
    valid = np.stack([k > 0, j > 0, i > 0, np.ones(N, bool), i < side - 1, j < side - 1, k < side - 1], axis=1)
    nb = node[:, None] + offs[None, :]                       # (N, 7) ascending neighbour ids
    nslots = valid.sum(axis=1).astype(np.int64)              # blocks per block-row
    per_row = dof * nslots                                   # entries per scalar row
    m = N * dof
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.repeat(per_row, dof), out=row_ptr[1:])
    # columns of one block-row: for each valid slot s, dof*nb[s] + e, e = 0..dof-1
    blockcols = (dof * nb[:, :, None] + np.arange(dof)[None, None, :])  # (N, 7, dof)
    vmask = np.broadcast_to(valid[:, :, None], blockcols.shape)
    rowcols = blockcols[vmask]                                # concatenated per node, len = per_row[node]
    del blockcols, vmask, nb
    # replicate each node's column list for its dof rows
    node_start = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(per_row, out=node_start[1:])
    # index of entry t of row (node, d): node_start[node] + t
    row_node = np.repeat(node, dof)
    lens = np.repeat(per_row, dof)
    starts = np.repeat(node_start[:-1], dof)
    off = np.arange(row_ptr[-1], dtype=np.int64) - np.repeat(row_ptr[:-1], lens)
    col = rowcols[np.repeat(starts, lens) + off].astype(np.int32)
    del rowcols, off
    val = _rng(seed, STREAM_MATRIX).uniform(-1.0, 1.0, size=col.shape[0])
    # scalar diagonal: self slot comes after the valid lower neighbours
    d = np.tile(np.arange(dof), N)
    lower = np.repeat((k > 0).astype(np.int64) + (j > 0) + (i > 0), dof)
    diag_pos = row_ptr[:-1] + dof * lower + d
    val[diag_pos] += shift
    del row_node
    return Csr(m, m, row_ptr, col, val, f"block3d_{side}x{dof}")


def zipf_truncated(rng: np.random.Generator, size: int, a: float, hi: int) -> np.ndarray:
    """Zipf(a) samples conditioned on [1, hi] (rejection of draws above hi)."""
    z = rng.zipf(a, size=size)
    bad = z > hi
    while bad.any():
        z[bad] = rng.zipf(a, size=int(bad.sum()))
        bad = z > hi
    return z.astype(np.int64)


def power_law(n: int = 4_000_000, seed: int = 2, a: float = 2.1, max_len: int = 100_000,
              mean_len: float | None = 16.0, local_frac: float = 0.7, window: int = 2048) -> Csr:
    """Square n x n matrix with power-law row lengths.

    Row lengths: Z ~ Zipf(a) truncated to [1, max_len]; the truncated law has a
    mean near 4.8 for a = 2.1, so when ``mean_len`` is given the lengths are
    L = min(max_len, n, round(s * Z)) with the scale s chosen (bisection on this
    sample) so that mean(L) is as close as possible to ``mean_len``; with
    ``mean_len=None`` the unscaled lengths are used.  Each row draws
    Binomial(L, local_frac) distinct columns inside [i - window, i + window]
    (capped at the window size) and the rest uniformly over [0, n), all
    distinct; columns are sorted; values are U[-1, 1]."""
    rng = _rng(seed, STREAM_MATRIX)
    z = zipf_truncated(rng, n, a, max_len)
    cap = min(max_len, n)
    if mean_len is None:
        L = np.minimum(z, cap)
        scale = 1.0
    else:
        lo_s, hi_s = 0.5, 64.0
        for _ in range(60):
            s = 0.5 * (lo_s + hi_s)
            mean = np.minimum(np.rint(s * z), cap).mean()
            if mean < mean_len:
                lo_s = s
            else:
                hi_s = s
        scale = 0.5 * (lo_s + hi_s)
        L = np.minimum(np.rint(scale * z), cap).astype(np.int64)
        L = np.maximum(L, 1)
    rows = np.arange(n, dtype=np.int64)
    wlo = np.maximum(rows - window, 0)
    whi = np.minimum(rows + window, n - 1)
    wsize = whi - wlo + 1
    nloc = np.minimum(rng.binomial(L, local_frac), wsize)
    nuni = L - nloc
    # local draws
    rl = np.repeat(rows, nloc)
    cl = wlo[rl] + (rng.random(rl.shape[0]) * wsize[rl]).astype(np.int64)
    ru = np.repeat(rows, nuni)
    cu = (rng.random(ru.shape[0]) * n).astype(np.int64)
    keys = np.unique(np.concatenate([rl * n + cl, ru * n + cu]))
    del rl, cl, ru, cu
    # rows whose distinct count fell short (duplicates) draw more: local rows that are
    # saturated cannot gain local columns, so all refills are uniform over [0, n).  Each
    # round adds the new distinct keys to the sorted set by insertion (the same set as a
    # unique() of the union, without re-sorting all keys).
    cnt = np.bincount(keys // n, minlength=n)
    for _ in range(1000):
        short = L - cnt
        if not (short > 0).any():
            break
        rr = np.repeat(rows, np.maximum(short, 0))
        cc = (rng.random(rr.shape[0]) * n).astype(np.int64)
        new = np.unique(rr * n + cc)
        pos = np.searchsorted(keys, new)
        fresh = pos >= keys.shape[0]
        fresh[~fresh] = keys[pos[~fresh]] != new[~fresh]
        new, pos = new[fresh], pos[fresh]
        keys = np.insert(keys, pos, new)
        cnt += np.bincount(new // n, minlength=n)
    else:  # pragma: no cover
        raise RuntimeError("power_law: could not fill rows")
    r = keys // n
    col = (keys % n).astype(np.int32)
    del keys
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=row_ptr[1:])
    val = rng.uniform(-1.0, 1.0, size=col.shape[0])
    out = Csr(n, n, row_ptr, col, val, f"powerlaw_{n}")
    out.scale = scale  # type: ignore[attr-defined]
    return out


def random_csr(m: int, n: int, density: float, seed: int, values: str = "uniform") -> Csr:
    """Uniformly random pattern (each entry present with probability ``density``).

    values: "uniform" U[-1,1]; "dyadic" p/64 with |p| <= 64 (exact products and
    sums in FP64); "int" small integers in [-8, 8]."""
    rng = _rng(seed, STREAM_MATRIX)
    if m == 0 or n == 0:
        return Csr(m, n, np.zeros(m + 1, np.int64), np.zeros(0, np.int32), np.zeros(0), "random")
    if m * n <= 4_000_000:
        mask = rng.random((m, n)) < density
        r, c = np.nonzero(mask)
    else:
        cnt = rng.binomial(n, density, size=m)
        rr = np.repeat(np.arange(m, dtype=np.int64), cnt)
        cc = (rng.random(rr.shape[0]) * n).astype(np.int64)
        keys = np.unique(rr * n + cc)
        r, c = keys // n, keys % n
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=m), out=row_ptr[1:])
    nnz = r.shape[0]
    if values == "uniform":
        val = rng.uniform(-1.0, 1.0, nnz)
    elif values == "dyadic":
        val = rng.integers(-64, 65, nnz).astype(np.float64) / 64.0
    elif values == "int":
        val = rng.integers(-8, 9, nnz).astype(np.float64)
    else:
        raise ValueError(values)
    return Csr(m, n, row_ptr, c.astype(np.int32), val, "random")


def from_dense(D: np.ndarray, keep_zeros_mask: np.ndarray | None = None) -> Csr:
    """CSR of a dense array; entries where ``keep_zeros_mask`` is True are stored
    even when zero (explicit zeros)."""
    D = np.asarray(D, dtype=np.float64)
    m, n = D.shape
    mask = D != 0
    if keep_zeros_mask is not None:
        mask |= keep_zeros_mask
    mask |= np.isnan(D)
    r, c = np.nonzero(mask)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=m), out=row_ptr[1:])
    return Csr(m, n, row_ptr, c.astype(np.int32), D[r, c].copy(), "dense")


def identity(n: int) -> Csr:
    return Csr(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), np.ones(n), "identity")


def permutation(n: int, seed: int) -> tuple[Csr, np.ndarray]:
    """P with P[i, pi[i]] = 1, so (P x)_i = x[pi[i]]."""
    pi = _rng(seed, STREAM_MATRIX).permutation(n).astype(np.int32)
    return Csr(n, n, np.arange(n + 1, dtype=np.int64), pi, np.ones(n), "permutation"), pi


def single_tile(nnz: int, seed: int, rows: int = 16, cols: int = 16) -> Csr:
    """A rows x cols matrix (one 16x16 tile) with exactly ``nnz`` entries at random
    distinct positions, values U[-1,1]."""
    rng = _rng(seed, STREAM_MATRIX)
    pos = np.sort(rng.choice(rows * cols, size=nnz, replace=False))
    r, c = pos // cols, pos % cols
    row_ptr = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=rows), out=row_ptr[1:])
    return Csr(rows, cols, row_ptr, c.astype(np.int32), rng.uniform(-1, 1, nnz), f"tile{nnz}")


def vector(n: int, seed: int, stream: int = STREAM_X, dyadic: bool = False) -> np.ndarray:
    """x ~ U[-1, 1] (or q/64 with |q| <= 64 when ``dyadic``)."""
    rng = _rng(seed, stream)
    if dyadic:
        return rng.integers(-64, 65, n).astype(np.float64) / 64.0
    return rng.uniform(-1.0, 1.0, n)


def rhs(n: int, k: int, seed: int) -> np.ndarray:
    """Row-major n x k block of right-hand sides, U[-1, 1]."""
    return _rng(seed, STREAM_RHS).uniform(-1.0, 1.0, size=(n, k))


def rhs_columns(n: int, k: int, seed0: int) -> np.ndarray:
    """Row-major n x k block whose column j is U[-1, 1] drawn from seed seed0 + j (so the first
    columns of a wider block are the same vectors)."""
    X = np.empty((n, k))
    for j in range(k):
        X[:, j] = _rng(seed0 + j, STREAM_RHS).uniform(-1.0, 1.0, n)
    return X
