// What the library's other native parts (the serving loop) read from a handle.  Internal to
// libcbspmv.
#pragma once

#include <cstdint>

#include "cb_device.h"
#include "cbspmv.h"

namespace cbh {

struct MatrixView {
    cbd::DevView view;   // device structure
    int kernel_vt = 0;   // kernel value code (cb_device.h)
    int vtype = 0;       // storage precision (cb_value_t)
    int vector_f64 = 1;  // x and y are double
    int col_agg = 0;     // the device view's: 0 none, 1 4-byte columns, 2 and 3 2-byte column offsets
    int row_reduce = 0;
    int natural = 1;     // natural-order structure (the streaming kernel)
    int device = -1;
    int64_t m = 0, n = 0, nnz = 0;
    int64_t nprepass = 0;
    int64_t device_bytes = 0;
};

// CB_ERROR_INVALID_VALUE for NULL, CB_ERROR_NOT_SUPPORTED for host-only handles.
cb_status_t matrix_view(cb_matrix_t A, MatrixView &out);

}  // namespace cbh
