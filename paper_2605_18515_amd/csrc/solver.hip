// Conjugate gradient on CB matrices (symmetric positive definite A), and FP64
// iterative refinement around a CG on a low-precision copy of the matrix.
//
// Every iteration runs on the device: the product through cb_spmv, the dot
// products as deterministic two-stage reductions accumulated in FP64, and the
// step lengths computed by the kernels from device scalars, so the host only
// reads the residual norm every check_every iterations.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "cb_host.h"
#include "cbspmv.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 1024;  // partial sums of one dot product

// device scalars of one CG solve
struct Scal {
    double rr;    // r.r of the current residual
    double pq;    // p.(A p)
    double rrn;   // r.r after the update
    double bb;    // b.b
    int32_t bad;  // p.(A p) <= 0 or not finite: A is not positive definite along p
    int32_t pad;
};

int blocks_for(int64_t n) {
    const int64_t b = (n + kThreads - 1) / kThreads;
    return (int)(b < kMaxBlocks ? (b < 1 ? 1 : b) : kMaxBlocks);
}

__device__ double block_sum(double v) {
    __shared__ double sh[kThreads / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kThreads / 64; ++i) s += sh[i];
    return s;
}

// partial[block] = sum over the block's grid-stride share of a[i] * b[i]
template <class T>
__global__ __launch_bounds__(kThreads) void dot_kernel(const T *__restrict__ a, const T *__restrict__ b, int64_t n,
                                                       double *__restrict__ partial) {
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        v += (double)a[i] * (double)b[i];
    const double s = block_sum(v);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// *dst = sum of the partials (fixed order); first, if given, *from is copied into *to
__global__ __launch_bounds__(64) void reduce_kernel(const double *__restrict__ partial, int g, double *dst,
                                                    const double *from, double *to) {
    double v = 0.0;
    for (int i = threadIdx.x; i < g; i += 64) v += partial[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if (threadIdx.x == 0) {
        if (from) *to = *from;
        *dst = v;
    }
}

// x += alpha p, r -= alpha q with alpha = rr / pq; partial sums of the new r.r
template <class T>
__global__ __launch_bounds__(kThreads) void update_xr_kernel(T *__restrict__ x, T *__restrict__ r,
                                                             const T *__restrict__ p, const T *__restrict__ q,
                                                             int64_t n, Scal *s, double *__restrict__ partial) {
    const double pq = s->pq;
    const bool ok = pq > 0.0 && std::isfinite(pq);
    if (!ok && blockIdx.x == 0 && threadIdx.x == 0) s->bad = 1;
    const T alpha = ok ? (T)(s->rr / pq) : T(0);
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        x[i] += alpha * p[i];
        const T ri = r[i] - alpha * q[i];
        r[i] = ri;
        v += (double)ri * (double)ri;
    }
    const double sum = block_sum(v);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

// p = r + beta p with beta = rrn / rr
template <class T>
__global__ __launch_bounds__(kThreads) void update_p_kernel(T *__restrict__ p, const T *__restrict__ r, int64_t n,
                                                            const Scal *s) {
    const T beta = s->rr > 0.0 ? (T)(s->rrn / s->rr) : T(0);
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        p[i] = r[i] + beta * p[i];
}

__global__ void clear_scal_kernel(Scal *s) {
    if (threadIdx.x == 0) *s = Scal{};
}

template <class T>
__global__ __launch_bounds__(kThreads) void fill_kernel(T *__restrict__ a, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) a[i] = v;
}

template <class T>
__global__ __launch_bounds__(kThreads) void copy_kernel(T *__restrict__ dst, const T *__restrict__ src, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        dst[i] = src[i];
}

// dst = (TL)(src * scale) in the inner solve's precision
template <class TL>
__global__ __launch_bounds__(kThreads) void scale_to_kernel(TL *__restrict__ dst, const double *__restrict__ src,
                                                            int64_t n, const double *__restrict__ rr) {
    const double nrm = sqrt(*rr);
    const double sc = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        dst[i] = (TL)(src[i] * sc);
}

// x += norm(r) * d (the inner solve ran on r / norm(r))
template <class TL>
__global__ __launch_bounds__(kThreads) void add_scaled_kernel(double *__restrict__ x, const TL *__restrict__ d,
                                                              int64_t n, const double *__restrict__ rr) {
    const double nrm = sqrt(*rr);
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        x[i] += nrm * (double)d[i];
}

cb_status_t fail(cb_status_t st, const std::string &msg) {
    cbh::set_last_error(msg);
    return st;
}

cb_status_t hipcheck(hipError_t e, const char *what) {
    if (e == hipSuccess) return CB_SUCCESS;
    return fail(CB_ERROR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct Mat {
    int64_t n = 0;
    int vtype = 0;
    int esize = 8;
};

cb_status_t mat_of(cb_matrix_t A, Mat &M) {
    if (!A) return fail(CB_ERROR_INVALID_VALUE, "NULL matrix handle");
    cb_info_t info{};
    info.struct_size = sizeof(cb_info_t);
    const cb_status_t st = cb_get_info(A, &info);
    if (st != CB_SUCCESS) return st;
    if (!info.on_device) return fail(CB_ERROR_NOT_SUPPORTED, "host-only handle (cb_create_host) cannot be solved with");
    if (info.m != info.n) return fail(CB_ERROR_INVALID_VALUE, "CG needs a square matrix");
    M.n = info.n;
    M.vtype = info.value_type;
    M.esize = info.value_type == CB_VALUE_F64 ? 8 : 4;
    return CB_SUCCESS;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// workspace of one CG solve with elements of esize bytes: r, p, q, partial sums, scalars
size_t cg_bytes(int64_t n, int esize) {
    return 3 * align256((size_t)n * esize) + align256(sizeof(double) * kMaxBlocks) + align256(sizeof(Scal));
}

// refinement: an FP64 solve's block, an FP32 solve's block, the inner right-hand side and solution
size_t refine_bytes(int64_t n) { return cg_bytes(n, 8) + cg_bytes(n, 4) + 2 * align256((size_t)n * 4); }

template <class T>
struct CgWork {
    T *r, *p, *q;
    double *partial;
    Scal *s;
};

template <class T>
CgWork<T> carve(void *work, int64_t n) {
    uint8_t *w = static_cast<uint8_t *>(work);
    CgWork<T> c;
    const size_t v = align256((size_t)n * sizeof(T));
    c.r = reinterpret_cast<T *>(w);
    c.p = reinterpret_cast<T *>(w + v);
    c.q = reinterpret_cast<T *>(w + 2 * v);
    c.partial = reinterpret_cast<double *>(w + 3 * v);
    c.s = reinterpret_cast<Scal *>(w + 3 * v + align256(sizeof(double) * kMaxBlocks));
    return c;
}

template <class T>
cb_status_t dot(const T *a, const T *b, int64_t n, double *partial, double *dst, hipStream_t st,
                const double *from = nullptr, double *to = nullptr) {
    const int g = blocks_for(n);
    hipLaunchKernelGGL(dot_kernel<T>, dim3(g), dim3(kThreads), 0, st, a, b, n, partial);
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(64), 0, st, partial, g, dst, from, to);
    return hipcheck(hipGetLastError(), "dot product launch");
}

cb_status_t read_scal(const Scal *s, Scal &h, hipStream_t st) {
    cb_status_t e = hipcheck(hipMemcpyAsync(&h, s, sizeof(Scal), hipMemcpyDeviceToHost, st), "scalar read");
    if (e != CB_SUCCESS) return e;
    return hipcheck(hipStreamSynchronize(st), "stream synchronize");
}

// CG on A x = b from the caller's x, elements T matching A's storage; stops when the recurrence
// residual is at most rtol * |b|.  Returns iterations, convergence, and |r|/|b| of the recurrence.
template <class T>
cb_status_t cg_solve(cb_matrix_t A, int64_t n, const T *b, T *x, const CgWork<T> &w, double rtol, int max_iter,
                     int check_every, hipStream_t st, int &iters, bool &converged, double &rel) {
    iters = 0;
    converged = false;
    const int g = blocks_for(n);
    cb_status_t e;
    hipLaunchKernelGGL(copy_kernel<T>, dim3(g), dim3(kThreads), 0, st, w.r, b, n);
    if ((e = cb_spmv(A, -1.0, x, 1.0, w.r, st)) != CB_SUCCESS) return e;
    hipLaunchKernelGGL(copy_kernel<T>, dim3(g), dim3(kThreads), 0, st, w.p, w.r, n);
    hipLaunchKernelGGL(clear_scal_kernel, dim3(1), dim3(64), 0, st, w.s);
    if ((e = dot<T>(b, b, n, w.partial, &w.s->bb, st)) != CB_SUCCESS) return e;
    if ((e = dot<T>(w.r, w.r, n, w.partial, &w.s->rr, st)) != CB_SUCCESS) return e;
    // the first residual norm also covers x already being the solution
    if ((e = dot<T>(w.r, w.r, n, w.partial, &w.s->rrn, st)) != CB_SUCCESS) return e;
    Scal h{};
    if ((e = read_scal(w.s, h, st)) != CB_SUCCESS) return e;
    const double target = rtol * std::sqrt(h.bb);
    rel = h.bb > 0.0 ? std::sqrt(h.rrn / h.bb) : std::sqrt(h.rrn);
    if (std::sqrt(h.rrn) <= target) {
        converged = true;
        return CB_SUCCESS;
    }
    for (int it = 1; it <= max_iter; ++it) {
        if ((e = cb_spmv(A, 1.0, w.p, 0.0, w.q, st)) != CB_SUCCESS) return e;
        // pq = p.q, and rr <- rrn from the previous iteration (the first has rr set already)
        if ((e = dot<T>(w.p, w.q, n, w.partial, &w.s->pq, st, it > 1 ? &w.s->rrn : nullptr,
                        it > 1 ? &w.s->rr : nullptr)) != CB_SUCCESS)
            return e;
        hipLaunchKernelGGL(update_xr_kernel<T>, dim3(g), dim3(kThreads), 0, st, x, w.r, w.p, w.q, n, w.s, w.partial);
        hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(64), 0, st, w.partial, g, &w.s->rrn, nullptr, nullptr);
        hipLaunchKernelGGL(update_p_kernel<T>, dim3(g), dim3(kThreads), 0, st, w.p, w.r, n, w.s);
        if ((e = hipcheck(hipGetLastError(), "CG step launch")) != CB_SUCCESS) return e;
        iters = it;
        if (it % check_every == 0 || it == max_iter) {
            if ((e = read_scal(w.s, h, st)) != CB_SUCCESS) return e;
            rel = h.bb > 0.0 ? std::sqrt(h.rrn / h.bb) : std::sqrt(h.rrn);
            if (std::sqrt(h.rrn) <= target) {
                converged = true;
                return CB_SUCCESS;
            }
            if (h.bad) return CB_SUCCESS;  // not positive definite along a search direction
        }
    }
    return CB_SUCCESS;
}

// |b - A x| / |b| in FP64 with the workspace's r as scratch
cb_status_t true_residual(cb_matrix_t A, int64_t n, const double *b, const double *x, const CgWork<double> &w,
                          hipStream_t st, double &rel, double &rr, double &bb) {
    const int g = blocks_for(n);
    cb_status_t e;
    hipLaunchKernelGGL(copy_kernel<double>, dim3(g), dim3(kThreads), 0, st, w.r, b, n);
    if ((e = cb_spmv(A, -1.0, x, 1.0, w.r, st)) != CB_SUCCESS) return e;
    if ((e = dot<double>(w.r, w.r, n, w.partial, &w.s->rr, st)) != CB_SUCCESS) return e;
    if ((e = dot<double>(b, b, n, w.partial, &w.s->bb, st)) != CB_SUCCESS) return e;
    Scal h{};
    if ((e = read_scal(w.s, h, st)) != CB_SUCCESS) return e;
    rr = h.rr;
    bb = h.bb;
    rel = bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    return CB_SUCCESS;
}

cb_status_t check_opts(const cb_cg_options_t *opt, cb_cg_options_t &o) {
    cb_cg_options_default(&o);
    if (!opt) return CB_SUCCESS;
    if (opt->struct_size != sizeof(cb_cg_options_t)) return fail(CB_ERROR_INVALID_VALUE, "cb_cg_options_t.struct_size mismatch");
    o = *opt;
    if (o.max_iter < 1 || o.check_every < 1 || o.max_refine < 1 || !(o.rtol >= 0.0) || !(o.inner_rtol > 0.0) ||
        !(o.inner_rtol < 1.0))
        return fail(CB_ERROR_INVALID_VALUE, "invalid CG options");
    return CB_SUCCESS;
}

}  // namespace

extern "C" {

cb_status_t cb_cg_options_default(cb_cg_options_t *opt) {
    if (!opt) return fail(CB_ERROR_INVALID_VALUE, "NULL options");
    *opt = cb_cg_options_t{};
    opt->struct_size = sizeof(cb_cg_options_t);
    opt->max_iter = 10000;
    opt->rtol = 1e-10;
    opt->check_every = 16;
    opt->max_refine = 50;
    opt->inner_rtol = 1e-4;
    return CB_SUCCESS;
}

cb_status_t cb_cg_workspace_bytes(cb_matrix_t A, cb_matrix_t A_low, int64_t *bytes) {
    if (!bytes) return fail(CB_ERROR_INVALID_VALUE, "NULL output");
    Mat M;
    cb_status_t st = mat_of(A, M);
    if (st != CB_SUCCESS) return st;
    size_t b = cg_bytes(M.n, M.esize);
    if (A_low) {
        Mat L;
        if ((st = mat_of(A_low, L)) != CB_SUCCESS) return st;
        if (L.n != M.n) return fail(CB_ERROR_INVALID_VALUE, "the two matrices differ in size");
        b = refine_bytes(M.n);
    }
    *bytes = (int64_t)b;
    return CB_SUCCESS;
}

cb_status_t cb_cg(cb_matrix_t A, const void *b, void *x, void *work, int64_t work_bytes, const cb_cg_options_t *opt,
                  cb_cg_result_t *res, void *stream) {
    cb_cg_options_t o;
    cb_status_t st = check_opts(opt, o);
    if (st != CB_SUCCESS) return st;
    Mat M;
    if ((st = mat_of(A, M)) != CB_SUCCESS) return st;
    if (!res || (M.n > 0 && (!b || !x || !work))) return fail(CB_ERROR_INVALID_VALUE, "NULL argument");
    if (work_bytes < (int64_t)cg_bytes(M.n, M.esize)) return fail(CB_ERROR_INVALID_VALUE, "workspace too small");
    cb_cg_result_t r{};
    hipStream_t s = (hipStream_t)stream;
    if (M.n > 0) {
        int iters = 0;
        bool conv = false;
        double rel = 0.0;
        if (M.vtype == CB_VALUE_F64)
            st = cg_solve<double>(A, M.n, (const double *)b, (double *)x, carve<double>(work, M.n), o.rtol, o.max_iter,
                                  o.check_every, s, iters, conv, rel);
        else
            st = cg_solve<float>(A, M.n, (const float *)b, (float *)x, carve<float>(work, M.n), o.rtol, o.max_iter,
                                 o.check_every, s, iters, conv, rel);
        if (st != CB_SUCCESS) return st;
        r.converged = conv;
        r.iterations = iters;
        r.rel_residual = rel;
        if (M.vtype == CB_VALUE_F64) {
            // report the true residual of the returned x (the recurrence drifts from it)
            double rr = 0.0, bb = 0.0;
            if ((st = true_residual(A, M.n, (const double *)b, (const double *)x, carve<double>(work, M.n), s, rel, rr,
                                    bb)) != CB_SUCCESS)
                return st;
            r.rel_residual = rel;
        }
    } else {
        r.converged = 1;
    }
    *res = r;
    return CB_SUCCESS;
}

cb_status_t cb_cg_refine(cb_matrix_t A, cb_matrix_t A_low, const double *b, double *x, void *work, int64_t work_bytes,
                         const cb_cg_options_t *opt, cb_cg_result_t *res, void *stream) {
    cb_cg_options_t o;
    cb_status_t st = check_opts(opt, o);
    if (st != CB_SUCCESS) return st;
    Mat M, L;
    if ((st = mat_of(A, M)) != CB_SUCCESS) return st;
    if ((st = mat_of(A_low, L)) != CB_SUCCESS) return st;
    if (M.vtype != CB_VALUE_F64 || L.vtype == CB_VALUE_F64)
        return fail(CB_ERROR_INVALID_VALUE, "refinement needs an FP64 matrix and an FP32 or BF16 copy");
    if (L.n != M.n) return fail(CB_ERROR_INVALID_VALUE, "the two matrices differ in size");
    if (!res || (M.n > 0 && (!b || !x || !work))) return fail(CB_ERROR_INVALID_VALUE, "NULL argument");
    const size_t need = refine_bytes(M.n);
    if (work_bytes < (int64_t)need) return fail(CB_ERROR_INVALID_VALUE, "workspace too small");
    cb_cg_result_t r{};
    if (M.n == 0) {
        r.converged = 1;
        *res = r;
        return CB_SUCCESS;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = M.n;
    const int g = blocks_for(n);
    // workspace: the FP64 block (residual, scalars), the inner solve's block, its right-hand side and
    // its solution
    uint8_t *wb = static_cast<uint8_t *>(work);
    const CgWork<double> w64 = carve<double>(wb, n);
    const CgWork<float> w32 = carve<float>(wb + cg_bytes(n, 8), n);
    float *rhs32 = reinterpret_cast<float *>(wb + cg_bytes(n, 8) + cg_bytes(n, 4));
    float *dsol = reinterpret_cast<float *>(wb + cg_bytes(n, 8) + cg_bytes(n, 4) + align256((size_t)n * 4));
    double rel = 0.0, rr = 0.0, bb = 0.0;
    if ((st = true_residual(A, n, b, x, w64, s, rel, rr, bb)) != CB_SUCCESS) return st;
    int total = 0, outer = 0;
    const double target = o.rtol * std::sqrt(bb);
    while (std::sqrt(rr) > target && outer < o.max_refine) {
        // inner solve on r / |r| with d = 0 as its start
        hipLaunchKernelGGL(scale_to_kernel<float>, dim3(g), dim3(kThreads), 0, s, rhs32, w64.r, n, &w64.s->rr);
        hipLaunchKernelGGL(fill_kernel<float>, dim3(g), dim3(kThreads), 0, s, dsol, n, 0.0f);
        if ((st = hipcheck(hipGetLastError(), "refinement launch")) != CB_SUCCESS) return st;
        int it = 0;
        bool conv = false;
        double irel = 0.0;
        if ((st = cg_solve<float>(A_low, n, rhs32, dsol, w32, o.inner_rtol, o.max_iter, o.check_every, s, it, conv,
                                  irel)) != CB_SUCCESS)
            return st;
        total += it;
        ++outer;
        hipLaunchKernelGGL(add_scaled_kernel<float>, dim3(g), dim3(kThreads), 0, s, x, dsol, n, &w64.s->rr);
        if ((st = hipcheck(hipGetLastError(), "refinement launch")) != CB_SUCCESS) return st;
        const double prev = rr;
        if ((st = true_residual(A, n, b, x, w64, s, rel, rr, bb)) != CB_SUCCESS) return st;
        if (!(rr < prev)) break;  // no progress: the low-precision solve cannot reduce the residual further
    }
    r.converged = std::sqrt(rr) <= target;
    r.iterations = total;
    r.refinements = outer;
    r.rel_residual = rel;
    *res = r;
    return CB_SUCCESS;
}

}  // extern "C"
