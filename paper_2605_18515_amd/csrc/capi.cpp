// C ABI of libcbspmv: handle lifetime, device upload, launches, export.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cb_device.h"
#include "cb_host.h"
#include "cb_internal.h"
#include "cbspmv.h"

namespace {

thread_local std::string g_err;

}  // namespace

namespace cbh {
void set_last_error(const std::string &msg) { g_err = msg; }
}  // namespace cbh

namespace {

cb_status_t fail(cb_status_t st, const std::string &msg) {
    g_err = msg;
    return st;
}

cb_status_t hip_fail(hipError_t e, const char *what) {
    const cb_status_t st = (e == hipErrorOutOfMemory) ? CB_ERROR_OUT_OF_MEMORY : CB_ERROR_HIP;
    return fail(st, std::string(what) + ": " + hipGetErrorString(e));
}

// byte offsets of every array inside the single device allocation
struct Layout {
    size_t tile_row, tile_col, tile_nnz, tile_vp, tile_type, tile_ori, tile_xoff, payload, restore_cols, cols_offset, wave_ptr,
        quantum_ptr, panel_shared, prepass_list, batch_stream, batch_ptr, tile_cols, tile_rec, panel_tile,
        tile_cbase, tile_c16, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout make_layout(const cbh::HostStructure &s) {
    Layout L{};
    size_t off = 0;
    auto put = [&](size_t bytes) {
        const size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    const size_t NT = (size_t)s.ntiles;
    L.tile_row = put(4 * NT);
    L.tile_col = put(4 * NT);
    L.tile_nnz = put(4 * NT);
    L.tile_vp = put(8 * NT);
    L.tile_type = put(NT);
    L.tile_ori = put(4 * NT);
    L.tile_xoff = put(s.col_agg ? 4 * NT : 0);
    // the streaming kernel reads whole 1 KB chunks past the last tile and the last restore entry
    L.payload = put((size_t)s.payload_bytes + cbs::kPayloadPad);
    L.restore_cols = put(4 * (size_t)s.nrestore + cbs::kPayloadPad);
    L.cols_offset = put(s.col_agg ? 4 * ((size_t)s.npanels + 1) : 0);
    L.wave_ptr = put(4 * ((size_t)s.nwaves + 1));
    L.quantum_ptr = put(4 * ((size_t)s.nquanta + 1));
    L.panel_shared = put((size_t)s.npanels);
    L.prepass_list = put(4 * (size_t)s.nprepass);
    // the streaming kernel reads 17 records from the start of every batch
    const bool stream = cbh::streamed_lb(s.lb_mode), natural = cbh::natural_lb(s.lb_mode);
    L.batch_stream = put(stream ? 16 * ((size_t)s.nrecords + cbs::kStreamRecordPad) : 0);
    L.batch_ptr = put(stream ? 4 * ((size_t)s.nwaves + 1) : 0);
    L.tile_cols = put(stream && s.col_agg ? 4 * (size_t)s.blk * NT : 0);
    L.tile_rec = put(natural ? 16 * NT : 0);
    L.panel_tile = put(natural ? 4 * ((size_t)s.npanels + 1) : 0);
    L.tile_cbase = put(s.cols16 == 1 ? 4 * NT : 0);
    L.tile_c16 = put(s.cols16 ? 2 * (size_t)s.blk * NT : 0);
    L.total = off;
    return L;
}

}  // namespace

struct cb_matrix_s {
    cbh::HostStructure h;  // full structure for host handles; counts only once uploaded
    bool on_device = false;
    int device = -1;
    void *dbuf = nullptr;
    Layout L{};
    cbd::DevView view{};
};

namespace {

// kernel value code: storage precision, plus 2 for FP32/BF16 values with double vectors
int kernel_vtype(const cbh::HostStructure &h) { return h.vtype != CB_VALUE_F64 && h.vector_f64 ? h.vtype + 2 : h.vtype; }

cb_status_t check_options(const cb_options_t *opt, cb_options_t &o) {
    cb_options_default(&o);
    if (!opt) return CB_SUCCESS;
    if (opt->struct_size != sizeof(cb_options_t))
        return fail(CB_ERROR_INVALID_VALUE, "cb_options_t.struct_size does not match this library (use cb_options_default)");
    o = *opt;
    return CB_SUCCESS;
}

cb_status_t create_common(cb_matrix_t *out, int64_t m, int64_t n, int64_t nnz, const int64_t *row_ptr,
                          const int32_t *col_idx, const double *values, const cb_options_t *opt,
                          cb_matrix_s *&A) {
    if (!out) return fail(CB_ERROR_INVALID_VALUE, "out is NULL");
    cb_options_t o;
    cb_status_t st = check_options(opt, o);
    if (st != CB_SUCCESS) return st;
    A = new (std::nothrow) cb_matrix_s();
    if (!A) return fail(CB_ERROR_OUT_OF_MEMORY, "host allocation failed");
    std::string err;
    st = cbh::convert(m, n, nnz, row_ptr, col_idx, values, o, A->h, err);
    if (st != CB_SUCCESS) {
        delete A;
        A = nullptr;
        return fail(st, err);
    }
    return CB_SUCCESS;
}

template <class T>
void put_array(std::vector<uint8_t> &stage, size_t at, const std::vector<T> &v) {
    if (!v.empty()) std::memcpy(stage.data() + at, v.data(), v.size() * sizeof(T));
}

template <class T>
const T *dptr(const cb_matrix_s *A, size_t at) {
    return reinterpret_cast<const T *>(static_cast<const uint8_t *>(A->dbuf) + at);
}

cb_status_t upload(cb_matrix_s *A, hipStream_t stream) {
    cbh::HostStructure &s = A->h;
    hipError_t e = hipGetDevice(&A->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    A->L = make_layout(s);
    const Layout &L = A->L;
    if (L.total > 0) {
        std::vector<uint8_t> stage;
        try {
            stage.assign(L.total, 0);
        } catch (const std::bad_alloc &) {
            return fail(CB_ERROR_OUT_OF_MEMORY, "host staging allocation failed");
        }
        put_array(stage, L.tile_row, s.tile_row);
        put_array(stage, L.tile_col, s.tile_col);
        put_array(stage, L.tile_nnz, s.tile_nnz);
        put_array(stage, L.tile_vp, s.tile_vp);
        put_array(stage, L.tile_type, s.tile_type);
        put_array(stage, L.tile_ori, s.tile_ori);
        put_array(stage, L.tile_xoff, s.tile_xoff);
        put_array(stage, L.payload, s.payload);
        put_array(stage, L.restore_cols, s.restore_cols);
        put_array(stage, L.cols_offset, s.cols_offset);
        put_array(stage, L.wave_ptr, s.wave_ptr);
        put_array(stage, L.quantum_ptr, s.quantum_ptr);
        put_array(stage, L.panel_shared, s.panel_shared);
        put_array(stage, L.prepass_list, s.prepass_list);
        put_array(stage, L.batch_stream, s.batch_stream);
        put_array(stage, L.batch_ptr, s.batch_ptr);
        put_array(stage, L.tile_cols, s.tile_cols);
        put_array(stage, L.tile_rec, s.tile_rec);
        put_array(stage, L.panel_tile, s.panel_tile);
        put_array(stage, L.tile_cbase, s.tile_cbase);
        put_array(stage, L.tile_c16, s.tile_c16);
        e = hipMalloc(&A->dbuf, L.total);
        if (e != hipSuccess) {
            A->dbuf = nullptr;
            return hip_fail(e, "hipMalloc of the matrix structure");
        }
        // the whole structure moves to the device in one transfer (Section 3.2)
        e = hipMemcpyAsync(A->dbuf, stage.data(), L.total, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "structure upload");
    }
    const bool streamed = cbh::streamed_lb(s.lb_mode);
    cbd::DevView &v = A->view;
    v.tile_row = dptr<int32_t>(A, L.tile_row);
    v.tile_col = dptr<int32_t>(A, L.tile_col);
    v.tile_nnz = dptr<int32_t>(A, L.tile_nnz);
    v.tile_vp = dptr<int64_t>(A, L.tile_vp);
    v.tile_type = dptr<uint8_t>(A, L.tile_type);
    v.tile_xoff = dptr<int32_t>(A, L.tile_xoff);
    v.payload = dptr<uint8_t>(A, L.payload);
    v.restore_cols = dptr<int32_t>(A, L.restore_cols);
    v.cols_offset = dptr<int32_t>(A, L.cols_offset);
    v.wave_ptr = dptr<int32_t>(A, L.wave_ptr);
    v.panel_shared = dptr<uint8_t>(A, L.panel_shared);
    v.prepass_list = dptr<int32_t>(A, L.prepass_list);
    v.batch_stream = dptr<int32_t>(A, L.batch_stream);
    v.batch_ptr = dptr<int32_t>(A, L.batch_ptr);
    v.tile_cols = dptr<int32_t>(A, L.tile_cols);
    v.tile_rec = dptr<int32_t>(A, L.tile_rec);
    v.panel_tile = dptr<int32_t>(A, L.panel_tile);
    v.tile_cbase = dptr<int32_t>(A, L.tile_cbase);
    v.tile_c16 = dptr<uint16_t>(A, L.tile_c16);
    v.m = s.m;
    v.n = s.n;
    v.nwaves = (int32_t)s.nwaves;
    v.npanels = (int32_t)s.npanels;
    v.nprepass = (int32_t)s.nprepass;
    v.col_agg = !s.col_agg ? 0 : s.cols16 == 2 ? 3 : s.cols16 == 1 ? 2 : 1;
    v.natural_order = cbh::natural_lb(s.lb_mode) ? 1 : 0;
    v.scatter = s.lb_mode == CB_LB_PAPER_STREAM ? 1 : 0;
    v.row_reduce = s.row_reduce;
    v.spmv_kernel = s.spmv_kernel;
    v.tile_lt = s.lt;
    v.xcd_chunk = s.xcd_chunk;
    v.payload_alloc = (int64_t)s.payload_bytes + cbs::kPayloadPad;
    v.stream_alloc = streamed ? 16 * ((int64_t)s.nrecords + cbs::kStreamRecordPad) : 0;
    // the device copy is the structure from now on
    std::vector<int32_t>().swap(s.tile_row);
    std::vector<int32_t>().swap(s.tile_col);
    std::vector<int32_t>().swap(s.tile_nnz);
    std::vector<int32_t>().swap(s.tile_ori);
    std::vector<int32_t>().swap(s.tile_xoff);
    std::vector<int64_t>().swap(s.tile_vp);
    std::vector<uint8_t>().swap(s.tile_type);
    std::vector<uint8_t>().swap(s.payload);
    std::vector<int32_t>().swap(s.restore_cols);
    std::vector<int32_t>().swap(s.cols_offset);
    std::vector<int32_t>().swap(s.quantum_ptr);
    std::vector<int32_t>().swap(s.wave_ptr);
    std::vector<uint8_t>().swap(s.panel_shared);
    std::vector<int32_t>().swap(s.prepass_list);
    std::vector<int32_t>().swap(s.batch_stream);
    std::vector<int32_t>().swap(s.batch_ptr);
    std::vector<int32_t>().swap(s.tile_cols);
    std::vector<int32_t>().swap(s.tile_rec);
    std::vector<int32_t>().swap(s.panel_tile);
    std::vector<int32_t>().swap(s.tile_cbase);
    std::vector<uint16_t>().swap(s.tile_c16);
    A->on_device = true;
    return CB_SUCCESS;
}

template <class T>
cb_status_t fetch(const cb_matrix_s *A, size_t at, size_t count, std::vector<T> &dst) {
    dst.resize(count);
    if (count == 0) return CB_SUCCESS;
    hipError_t e = hipMemcpy(dst.data(), dptr<uint8_t>(A, at), count * sizeof(T), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "structure download");
    return CB_SUCCESS;
}

// host copy of the structure: the handle's own for host handles, downloaded otherwise
cb_status_t host_view(const cb_matrix_s *A, cbh::HostStructure &tmp, const cbh::HostStructure *&s) {
    if (!A->on_device) {
        s = &A->h;
        return CB_SUCCESS;
    }
    tmp = A->h;
    const Layout &L = A->L;
    const size_t NT = (size_t)A->h.ntiles;
    cb_status_t st;
    if ((st = fetch(A, L.tile_row, NT, tmp.tile_row)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.tile_col, NT, tmp.tile_col)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.tile_nnz, NT, tmp.tile_nnz)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.tile_vp, NT, tmp.tile_vp)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.tile_type, NT, tmp.tile_type)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.tile_ori, NT, tmp.tile_ori)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.tile_xoff, A->h.col_agg ? NT : 0, tmp.tile_xoff)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.payload, (size_t)A->h.payload_bytes, tmp.payload)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.restore_cols, (size_t)A->h.nrestore, tmp.restore_cols)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.cols_offset, A->h.col_agg ? (size_t)A->h.npanels + 1 : 0, tmp.cols_offset)) != CB_SUCCESS)
        return st;
    if ((st = fetch(A, L.wave_ptr, (size_t)A->h.nwaves + 1, tmp.wave_ptr)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.quantum_ptr, (size_t)A->h.nquanta + 1, tmp.quantum_ptr)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.panel_shared, (size_t)A->h.npanels, tmp.panel_shared)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.prepass_list, (size_t)A->h.nprepass, tmp.prepass_list)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.batch_stream, 4 * (size_t)A->h.nrecords, tmp.batch_stream)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.batch_ptr, cbh::streamed_lb(A->h.lb_mode) ? (size_t)A->h.nwaves + 1 : 0, tmp.batch_ptr)) !=
        CB_SUCCESS)
        return st;
    if ((st = fetch(A, L.tile_cols, cbh::streamed_lb(A->h.lb_mode) && A->h.col_agg ? (size_t)A->h.blk * NT : 0,
                    tmp.tile_cols)) != CB_SUCCESS)
        return st;
    if ((st = fetch(A, L.tile_cbase, A->h.cols16 == 1 ? NT : 0, tmp.tile_cbase)) != CB_SUCCESS) return st;
    if ((st = fetch(A, L.tile_c16, A->h.cols16 ? (size_t)A->h.blk * NT : 0, tmp.tile_c16)) != CB_SUCCESS) return st;
    s = &tmp;
    return CB_SUCCESS;
}

cb_status_t check_launch(const cb_matrix_s *A) {
    if (!A) return fail(CB_ERROR_INVALID_VALUE, "NULL matrix handle");
    if (!A->on_device) return fail(CB_ERROR_NOT_SUPPORTED, "host-only handle (cb_create_host) cannot run products");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != A->device) return fail(CB_ERROR_INVALID_VALUE, "the current device is not the device the matrix lives on");
    return CB_SUCCESS;
}

}  // namespace

extern "C" {

cb_status_t cb_options_default(cb_options_t *opt) {
    if (!opt) return fail(CB_ERROR_INVALID_VALUE, "opt is NULL");
    std::memset(opt, 0, sizeof(*opt));
    opt->struct_size = sizeof(cb_options_t);
    opt->value_type = CB_VALUE_F64;
    opt->col_agg = -1;
    opt->th1 = 32;
    opt->th2 = 128;
    opt->quantum_tiles = 8;
    opt->lb_mode = CB_LB_CONTIGUOUS;
    opt->host_threads = 0;
    opt->th0 = 0.15;
    opt->wave_nnz = 0;
    opt->row_reduce = -1;
    opt->spmv_kernel = -1;
    opt->xcd_chunk = -1;
    return CB_SUCCESS;
}

cb_status_t cb_create(cb_matrix_t *out, int64_t m, int64_t n, int64_t nnz, const int64_t *row_ptr,
                      const int32_t *col_idx, const double *values, const cb_options_t *opt, void *stream) {
    cb_matrix_s *A = nullptr;
    cb_status_t st = create_common(out, m, n, nnz, row_ptr, col_idx, values, opt, A);
    if (st != CB_SUCCESS) return st;
    st = upload(A, (hipStream_t)stream);
    if (st != CB_SUCCESS) {
        if (A->dbuf) (void)hipFree(A->dbuf);
        delete A;
        return st;
    }
    *out = A;
    return CB_SUCCESS;
}

cb_status_t cb_create_host(cb_matrix_t *out, int64_t m, int64_t n, int64_t nnz, const int64_t *row_ptr,
                           const int32_t *col_idx, const double *values, const cb_options_t *opt) {
    cb_matrix_s *A = nullptr;
    cb_status_t st = create_common(out, m, n, nnz, row_ptr, col_idx, values, opt, A);
    if (st != CB_SUCCESS) return st;
    *out = A;
    return CB_SUCCESS;
}

cb_status_t cb_destroy(cb_matrix_t A) {
    if (!A) return CB_SUCCESS;
    hipError_t e = hipSuccess;
    if (A->dbuf) e = hipFree(A->dbuf);
    delete A;
    if (e != hipSuccess) return hip_fail(e, "hipFree");
    return CB_SUCCESS;
}

cb_status_t cb_spmv(cb_matrix_t A, double alpha, const void *x, double beta, void *y, void *stream) {
    cb_status_t st = check_launch(A);
    if (st != CB_SUCCESS) return st;
    if (A->h.m > 0 && !y) return fail(CB_ERROR_INVALID_VALUE, "y is NULL");
    if (A->h.nnz > 0 && !x) return fail(CB_ERROR_INVALID_VALUE, "x is NULL");
    if (A->h.m == 0) return CB_SUCCESS;
    hipError_t e = cbd::launch_spmv(A->view, kernel_vtype(A->h), alpha, x, beta, y, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "cb_spmv launch");
    return CB_SUCCESS;
}

cb_status_t cb_spmm(cb_matrix_t A, int32_t k, double alpha, const void *X, int64_t ldx, double beta, void *Y,
                    int64_t ldy, void *stream) {
    cb_status_t st = check_launch(A);
    if (st != CB_SUCCESS) return st;
    if (k < 1) return fail(CB_ERROR_INVALID_VALUE, "k must be at least 1");
    if (ldx < k || ldy < k) return fail(CB_ERROR_INVALID_VALUE, "leading dimensions must be at least k");
    if (A->h.m > 0 && !Y) return fail(CB_ERROR_INVALID_VALUE, "Y is NULL");
    if (A->h.nnz > 0 && !X) return fail(CB_ERROR_INVALID_VALUE, "X is NULL");
    if (A->h.m == 0) return CB_SUCCESS;
    if (k == 1 && ldx == 1 && ldy == 1) return cb_spmv(A, alpha, X, beta, Y, stream);
    hipError_t e = cbd::launch_spmm(A->view, kernel_vtype(A->h), k, alpha, X, ldx, beta, Y, ldy, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "cb_spmm launch");
    return CB_SUCCESS;
}

cb_status_t cb_export_csr(cb_matrix_t A, int64_t *row_ptr, int32_t *col_idx, void *values) {
    if (!A) return fail(CB_ERROR_INVALID_VALUE, "NULL matrix handle");
    cbh::HostStructure tmp;
    const cbh::HostStructure *s = nullptr;
    cb_status_t st = host_view(A, tmp, s);
    if (st != CB_SUCCESS) return st;
    std::string err;
    st = cbh::export_csr(*s, row_ptr, col_idx, values, err);
    if (st != CB_SUCCESS) return fail(st, err);
    return CB_SUCCESS;
}

cb_status_t cb_get_info(cb_matrix_t A, cb_info_t *info) {
    if (!A || !info) return fail(CB_ERROR_INVALID_VALUE, "NULL argument");
    if (info->struct_size != sizeof(cb_info_t))
        return fail(CB_ERROR_INVALID_VALUE, "cb_info_t.struct_size does not match this library");
    cb_info_t out;
    std::memset(&out, 0, sizeof(out));
    out.struct_size = sizeof(cb_info_t);
    cbh::fill_info(A->h, out);
    out.on_device = A->on_device ? 1 : 0;
    out.device_bytes = A->on_device ? (int64_t)A->L.total : 0;
    *info = out;
    return CB_SUCCESS;
}

cb_status_t cb_export_structure(cb_matrix_t A, const cb_structure_t *o) {
    if (!A || !o) return fail(CB_ERROR_INVALID_VALUE, "NULL argument");
    cbh::HostStructure tmp;
    const cbh::HostStructure *s = nullptr;
    cb_status_t st = host_view(A, tmp, s);
    if (st != CB_SUCCESS) return st;
    auto cp = [](auto *dst, const auto &v) {
        if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    };
    cp(o->tile_row, s->tile_row);
    cp(o->tile_col, s->tile_col);
    cp(o->tile_nnz, s->tile_nnz);
    cp(o->tile_vp, s->tile_vp);
    cp(o->tile_type, s->tile_type);
    cp(o->tile_ori, s->tile_ori);
    cp(o->tile_xoff, s->tile_xoff);
    cp(o->payload, s->payload);
    cp(o->restore_cols, s->restore_cols);
    cp(o->cols_offset, s->cols_offset);
    cp(o->quantum_ptr, s->quantum_ptr);
    cp(o->wave_ptr, s->wave_ptr);
    cp(o->panel_shared, s->panel_shared);
    cp(o->prepass_list, s->prepass_list);
    cp(o->batch_stream, s->batch_stream);
    cp(o->batch_ptr, s->batch_ptr);
    cp(o->tile_cols, s->tile_cols);
    cp(o->tile_cbase, s->tile_cbase);
    cp(o->tile_c16, s->tile_c16);
    return CB_SUCCESS;
}

cb_status_t cb_copy_probe(const void *src, void *dst, int64_t bytes, void *stream) {
    if (bytes < 0 || (bytes & 15)) return fail(CB_ERROR_INVALID_VALUE, "bytes must be a non-negative multiple of 16");
    if (bytes == 0) return CB_SUCCESS;
    if (!src || !dst || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
        return fail(CB_ERROR_INVALID_VALUE, "src and dst must be non-NULL and 16-byte aligned");
    const uintptr_t s0 = (uintptr_t)src, d0 = (uintptr_t)dst;
    if (s0 < d0 + (uintptr_t)bytes && d0 < s0 + (uintptr_t)bytes)
        return fail(CB_ERROR_INVALID_VALUE, "src and dst overlap");
    hipError_t e = cbd::launch_copy(src, dst, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "cb_copy_probe launch");
    return CB_SUCCESS;
}

cb_status_t cb_read_probe(const void *src, int64_t bytes, void *sink, void *stream) {
    if (bytes < 0 || (bytes & 15)) return fail(CB_ERROR_INVALID_VALUE, "bytes must be a non-negative multiple of 16");
    if (bytes == 0) return CB_SUCCESS;
    if (!src || !sink || ((uintptr_t)src & 15) || ((uintptr_t)sink & 15))
        return fail(CB_ERROR_INVALID_VALUE, "src and sink must be non-NULL and 16-byte aligned");
    hipError_t e = cbd::launch_read(src, bytes, sink, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "cb_read_probe launch");
    return CB_SUCCESS;
}

const char *cb_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace cbh {

cb_status_t matrix_view(cb_matrix_t A, MatrixView &out) {
    if (!A) return fail(CB_ERROR_INVALID_VALUE, "NULL matrix handle");
    if (!A->on_device) return fail(CB_ERROR_NOT_SUPPORTED, "host-only handle (cb_create_host)");
    out.view = A->view;
    out.kernel_vt = kernel_vtype(A->h);
    out.vtype = A->h.vtype;
    out.vector_f64 = A->h.vector_f64;
    out.col_agg = A->view.col_agg;
    out.row_reduce = A->h.row_reduce;
    out.natural = cbh::natural_lb(A->h.lb_mode);
    out.device = A->device;
    out.m = A->h.m;
    out.n = A->h.n;
    out.nnz = A->h.nnz;
    out.nprepass = A->h.nprepass;
    out.device_bytes = (int64_t)A->L.total;
    return CB_SUCCESS;
}

}  // namespace cbh
