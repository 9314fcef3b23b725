"""CB-SpMV for AMD Instinct MI355X (gfx950).

The product is ``libcbspmv.so`` (C ABI declared in include/cbspmv.h): a host
converter from CSR to the CB tile structure and hand-written HIP kernels for
y = alpha*A*x + beta*y and its k-right-hand-side form.  ``cbspmv`` is the
ctypes binding (import it to load the library; it raises ImportError when the
library is not built), ``matgen`` the seeded synthetic matrices, ``build``
the in-tree build of the library.
"""
__all__ = ["cbspmv", "matgen", "build"]
