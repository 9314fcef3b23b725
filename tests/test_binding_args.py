"""Host-side checks of the Python binding's argument marshalling (no GPU): the C ABI takes every
vector as one unit-stride array and every k-right-hand-side block as rows of at least k elements,
so the binding refuses tensors whose memory does not have that shape before any pointer reaches
the library (a strided view would be read wrongly, an expanded one would be read or written past
its allocation)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2605_18515_amd import matgen

cb = pytest.importorskip("paper_2605_18515_amd.cbspmv", reason="libcbspmv.so not built")


@pytest.fixture
def host_matrix():
    A = matgen.laplacian_2d(8)
    M = cb.CbMatrix.from_csr(A, device=False)
    yield A, M
    M.close()


def test_expanded_vector_is_refused(host_matrix):
    A, M = host_matrix
    x = torch.zeros(1, dtype=torch.float64).expand(A.n)
    y = torch.zeros(A.m, dtype=torch.float64)
    with pytest.raises(ValueError, match="not contiguous"):
        M.spmv(x, y)
    with pytest.raises(ValueError, match="not contiguous"):
        M.spmv(y, x)


def test_column_view_is_refused(host_matrix):
    A, M = host_matrix
    base = torch.zeros((A.n, 3), dtype=torch.float64)
    col = base[:, 1]
    assert col.stride() == (3,)
    with pytest.raises(ValueError, match="not contiguous"):
        M.spmv(col, torch.zeros(A.m, dtype=torch.float64))
    with pytest.raises(ValueError, match="not contiguous"):
        M.spmv(torch.zeros(A.n, dtype=torch.float64), base[:, 2])


def test_strided_cg_vectors_are_refused(host_matrix):
    A, M = host_matrix
    b = torch.zeros(2 * A.n, dtype=torch.float64)[::2]
    with pytest.raises(ValueError, match="not contiguous"):
        M.cg(b, torch.zeros(A.n, dtype=torch.float64))


def test_spmm_rows_must_not_overlap(host_matrix):
    A, M = host_matrix
    k = 4
    X = torch.zeros((1, k), dtype=torch.float64).expand(A.n, k)  # row stride 0
    Y = torch.zeros((A.m, k), dtype=torch.float64)
    with pytest.raises(ValueError, match="rows overlap"):
        M.spmm(X, Y)
    with pytest.raises(ValueError, match="rows overlap"):
        M.spmm(torch.zeros((A.n, k), dtype=torch.float64), torch.zeros((1, k), dtype=torch.float64).expand(A.m, k))
    Xt = torch.zeros((k, A.n), dtype=torch.float64).t()  # column-major
    with pytest.raises(ValueError, match="row-major"):
        M.spmm(Xt, Y)


def test_server_host_vectors_must_be_contiguous():
    n = 10
    good = np.zeros(n)
    cb.check_host_vectors(np.float64, n, b=good, x=good.copy())
    strided = np.zeros(2 * n)[::2]
    with pytest.raises(ValueError, match="b must be C-contiguous"):
        cb.check_host_vectors(np.float64, n, b=strided, x=good)
    with pytest.raises(ValueError, match="x must be C-contiguous"):
        cb.check_host_vectors(np.float64, n, b=good, x=strided)
    with pytest.raises(ValueError, match="float32"):
        cb.check_host_vectors(np.float32, n, b=good, x=good)


def test_noalloc_cg_limit_and_host_handle():
    """The fixed workspace size of cb_cg_noalloc in the binding equals the header's, and a host-only
    handle or a NULL handle is refused before any device work."""
    import os
    import re

    text = open(os.path.join(os.path.dirname(cb.LIB_PATH), "..", "include", "cbspmv.h")).read()
    m = re.search(r"#define CB_CG_NOALLOC_MAX_BYTES \((\d+) \* (\d+) \* (\d+)\)", text)
    assert m and int(m[1]) * int(m[2]) * int(m[3]) == cb.CB_CG_NOALLOC_MAX_BYTES
    A = matgen.identity(20)
    h = cb.cb_create_host(20, 20, 20, A.row_ptr, A.col_idx, A.values)
    lib = cb.library_handle()
    r = cb.CbCgResult()
    assert lib.cb_cg_noalloc(h, 16, 32, None, ctypes.byref(r), None) == cb.CB_ERROR_NOT_SUPPORTED
    assert lib.cb_cg_noalloc(None, 16, 32, None, ctypes.byref(r), None) == cb.CB_ERROR_INVALID_VALUE
    cb.cb_destroy(h)
