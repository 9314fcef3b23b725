// Conjugate gradient on CB matrices (symmetric positive definite A), and two
// mixed-precision solvers that reach an FP64 residual while the products run on
// an FP32 or BF16 copy of the matrix.
//
// Every iteration runs on the device: the product through cb_spmv, the dot
// products accumulated in FP64 (block sums, then added in block order by a
// one-block kernel, or for p.q by every block of the update kernel that needs
// it, so results do not depend on timing; a last-block-done reduction inside
// the same kernel needs a device-scope fence per block, which writes back the
// XCD's L2 and measured slower), and the step lengths computed by the update
// kernels from device scalars.  The host reads the residual norm
// every check_every iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>

#include "cb_host.h"
#include "cb_internal.h"
#include "cbspmv.h"

// Workspace of cb_cg_noalloc: a fixed array in device memory, one copy per GPU the library runs on,
// held until the process ends.  Host code never passes this name to a kernel or a copy (on the host
// it is only a stand-in for the symbol); it uses the device address hipGetSymbolAddress returns for
// the current device.
static __device__ __align__(256) uint8_t scratch[CB_CG_NOALLOC_MAX_BYTES];

namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 1024;  // block sums of one reduction

// device scalars of one solve
struct Scal {
    double rr;       // r.r of the current residual
    double pq;       // p.(A p)
    double rrn;      // r.r after the update
    double bb;       // b.b
    int32_t bad;     // p.(A p) <= 0 or not finite: A is not positive definite along p
    int32_t pad;
};

int blocks_for(int64_t n) {
    const int64_t b = (n + kThreads - 1) / kThreads;
    return (int)(b < kMaxBlocks ? (b < 1 ? 1 : b) : kMaxBlocks);
}

// sum over the block, valid in thread 0
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

// partial[block] = the block's share of a.b (FP64 sums)
template <class TA, class TB>
__global__ __launch_bounds__(kThreads) void dot_kernel(const TA *__restrict__ a, const TB *__restrict__ b, int64_t n,
                                                       double *__restrict__ partial) {
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        v += (double)a[i] * (double)b[i];
    const double s = block_sum(v);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// *dst = the g block sums added in block order; first, when from is set, *to = *from
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

// x += alpha p, r -= alpha q with alpha = rr / pq (in FP64, rounded on store), where pq adds the g
// block sums of p.q (pq_part) in reduce_kernel's order, in every block, and rr is the r.r the
// previous step ended with (rrn); block sums of the new r.r (rr_part).  Block 0 records rr and pq
// for update_p_kernel and the host; no other block reads them here.
template <class TR, class TV>
__global__ __launch_bounds__(kThreads) void update_xr_kernel(TR *__restrict__ x, TR *__restrict__ r,
                                                             const TV *__restrict__ p, const TV *__restrict__ q,
                                                             int64_t n, Scal *s, const double *__restrict__ pq_part,
                                                             int g, double *__restrict__ rr_part) {
    __shared__ double tot;
    if (threadIdx.x < 64) {
        double v = 0.0;
        for (int i = threadIdx.x; i < g; i += 64) v += pq_part[i];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
        if (threadIdx.x == 0) tot = v;
    }
    __syncthreads();
    const double pq = tot;
    const double rr = s->rrn;
    const bool ok = pq > 0.0 && std::isfinite(pq);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s->rr = rr;
        s->pq = pq;
        if (!ok) s->bad = 1;
    }
    const double alpha = ok ? rr / pq : 0.0;
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        x[i] = (TR)((double)x[i] + alpha * (double)p[i]);
        const TR ri = (TR)((double)r[i] - alpha * (double)q[i]);
        r[i] = ri;
        v += (double)ri * (double)ri;
    }
    const double sum = block_sum(v);
    if (threadIdx.x == 0) rr_part[blockIdx.x] = sum;
}

// p = r + beta p with beta = rrn / rr
template <class TR, class TV>
__global__ __launch_bounds__(kThreads) void update_p_kernel(TV *__restrict__ p, const TR *__restrict__ r, int64_t n,
                                                            const Scal *s) {
    const double beta = s->rr > 0.0 ? s->rrn / s->rr : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        p[i] = (TV)((double)r[i] + beta * (double)p[i]);
}

__global__ void clear_scal_kernel(Scal *s) {
    if (threadIdx.x == 0) *s = Scal{};
}

template <class T>
__global__ __launch_bounds__(kThreads) void fill_kernel(T *__restrict__ a, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) a[i] = v;
}

// dst = (TD)src
template <class TD, class TS>
__global__ __launch_bounds__(kThreads) void copy_kernel(TD *__restrict__ dst, const TS *__restrict__ src, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        dst[i] = (TD)src[i];
}

// dst = (TL)(src / sqrt(*rr))
template <class TL>
__global__ __launch_bounds__(kThreads) void scale_to_kernel(TL *__restrict__ dst, const double *__restrict__ src,
                                                            int64_t n, const double *__restrict__ rr) {
    const double nrm = sqrt(*rr);
    const double sc = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        dst[i] = (TL)(src[i] * sc);
}

// x += sqrt(*rr) d
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
    int esize = 8;  // bytes of one vector element: 8 when x and y are double
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
    M.esize = info.vector_f64 ? 8 : 4;
    return CB_SUCCESS;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// workspace of one CG run: residual (sr bytes per element), direction and product (sv bytes),
// two sets of block sums (p.q, read by the update kernel, and r.r, which it writes), scalars
size_t cg_bytes(int64_t n, int sr, int sv) {
    return align256((size_t)n * sr) + 2 * align256((size_t)n * sv) + align256(sizeof(double) * 2 * kMaxBlocks) +
           align256(sizeof(Scal));
}

// restarted refinement: an FP64 block (true residual), the inner CG's block, its right-hand side and
// solution in the low-precision handle's vector type (esize bytes); the residual-replacement
// solver needs cg_bytes(n, 8, esize), which is smaller
size_t refine_bytes(int64_t n, int esize) {
    return cg_bytes(n, 8, 8) + cg_bytes(n, esize, esize) + 2 * align256((size_t)n * esize);
}

template <class TR, class TV>
struct Work {
    TR *r;
    TV *p, *q;
    double *partial, *partial2;
    Scal *s;
};

template <class TR, class TV>
Work<TR, TV> carve(void *work, int64_t n) {
    uint8_t *w = static_cast<uint8_t *>(work);
    Work<TR, TV> c;
    const size_t vr = align256((size_t)n * sizeof(TR)), vv = align256((size_t)n * sizeof(TV));
    c.r = reinterpret_cast<TR *>(w);
    c.p = reinterpret_cast<TV *>(w + vr);
    c.q = reinterpret_cast<TV *>(w + vr + vv);
    c.partial = reinterpret_cast<double *>(w + vr + 2 * vv);
    c.partial2 = c.partial + kMaxBlocks;
    c.s = reinterpret_cast<Scal *>(w + vr + 2 * vv + align256(sizeof(double) * 2 * kMaxBlocks));
    return c;
}

template <class TA, class TB>
void dot(const TA *a, const TB *b, int64_t n, double *partial, Scal *s, double *dst, hipStream_t st,
         const double *from = nullptr, double *to = nullptr) {
    (void)s;
    const int g = blocks_for(n);
    hipLaunchKernelGGL((dot_kernel<TA, TB>), dim3(g), dim3(kThreads), 0, st, a, b, n, partial);
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(64), 0, st, partial, g, dst, from, to);
}

cb_status_t read_scal(const Scal *s, Scal &h, hipStream_t st) {
    cb_status_t e = hipcheck(hipMemcpyAsync(&h, s, sizeof(Scal), hipMemcpyDeviceToHost, st), "scalar read");
    if (e != CB_SUCCESS) return e;
    return hipcheck(hipStreamSynchronize(st), "stream synchronize");
}

double rel_of(const Scal &h, double rr) { return h.bb > 0.0 ? std::sqrt(rr / h.bb) : std::sqrt(rr); }

// r = b - A x, vectors of A's type
template <class TR>
cb_status_t residual(cb_matrix_t A, int64_t n, const TR *b, const TR *x, TR *r, hipStream_t st) {
    hipLaunchKernelGGL((copy_kernel<TR, TR>), dim3(blocks_for(n)), dim3(kThreads), 0, st, r, b, n);
    return cb_spmv(A, -1.0, x, 1.0, r, st);
}

struct RunOut {
    int iters = 0;
    int replacements = 0;
    int restarts = 0;
    bool converged = false;
    double rel = 0.0;  // |r| / |b| of the last residual the solver holds (true after a replacement)
};

// CG on A x = b from the caller's x.  The residual r and iterate x are TR (b too); the direction p
// and the product q = Aop p are TV, Aop's vector type.  With Ahi set (TR = double, Aop stored in
// FP32 or BF16), the residual is replaced by the true FP64 residual b - Ahi x whenever the
// recurrence has fallen by replace_factor since the last replacement, and convergence is decided
// on the true residual only.  The direction is kept across a replacement (the Krylov space goes
// on) unless the true residual has not halved since the previous replacement, or the recurrence
// has gone eight checks without a new low (10 % below the last): then the low-precision
// operator's error has outgrown the recurrence and CG restarts from p = r.
// Without Ahi the recurrence decides.
template <class TR, class TV>
cb_status_t cg_run(cb_matrix_t Aop, cb_matrix_t Ahi, int64_t n, const TR *b, TR *x, const Work<TR, TV> &w,
                   double rtol, int max_iter, int check_every, double replace_factor, hipStream_t st, RunOut &out) {
    out = RunOut{};
    const int g = blocks_for(n);
    cb_status_t e;
    hipLaunchKernelGGL(clear_scal_kernel, dim3(1), dim3(64), 0, st, w.s);
    if ((e = residual<TR>(Ahi ? Ahi : Aop, n, b, x, w.r, st)) != CB_SUCCESS) return e;
    hipLaunchKernelGGL((copy_kernel<TV, TR>), dim3(g), dim3(kThreads), 0, st, w.p, w.r, n);
    dot(b, b, n, w.partial, w.s, &w.s->bb, st);
    dot(w.r, w.r, n, w.partial, w.s, &w.s->rr, st);
    dot(w.r, w.r, n, w.partial, w.s, &w.s->rrn, st);
    Scal h{};
    if ((e = read_scal(w.s, h, st)) != CB_SUCCESS) return e;
    const double target = rtol * std::sqrt(h.bb);
    double anchor = std::sqrt(h.rrn);  // true residual norm at the last replacement
    double best = anchor;
    int stalls = 0, low_it = 0;
    double low = anchor;  // lowest recurrence residual since the last replacement
    out.rel = rel_of(h, h.rrn);
    if (std::sqrt(h.rrn) <= target) {
        out.converged = true;
        return CB_SUCCESS;
    }
    for (int it = 1; it <= max_iter; ++it) {
        if ((e = cb_spmv(Aop, 1.0, w.p, 0.0, w.q, st)) != CB_SUCCESS) return e;
        // block sums of p.q; the update adds them itself and takes rr from the r.r the previous step
        // (or the start, or a replacement) left in rrn
        hipLaunchKernelGGL((dot_kernel<TV, TV>), dim3(g), dim3(kThreads), 0, st, w.p, w.q, n, w.partial);
        hipLaunchKernelGGL((update_xr_kernel<TR, TV>), dim3(g), dim3(kThreads), 0, st, x, w.r, w.p, w.q, n, w.s,
                           w.partial, g, w.partial2);
        hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(64), 0, st, w.partial2, g, &w.s->rrn, nullptr, nullptr);
        if ((e = hipcheck(hipGetLastError(), "CG step launch")) != CB_SUCCESS) return e;
        out.iters = it;
        if (it % check_every == 0 || it == max_iter) {
            if ((e = read_scal(w.s, h, st)) != CB_SUCCESS) return e;
            const double rn = std::sqrt(h.rrn);
            out.rel = rel_of(h, h.rrn);
            if (!Ahi) {
                if (rn <= target) {
                    out.converged = true;
                    return CB_SUCCESS;
                }
            } else if (rn < 0.9 * low) {
                low = rn;
                low_it = it;
            }
            if (Ahi && (rn <= target || rn <= replace_factor * anchor || it - low_it >= 8 * check_every)) {
                const bool stalled = rn > target && rn > replace_factor * anchor;
                // residual replacement: the true residual in FP64 takes the recurrence's place
                if ((e = residual<TR>(Ahi, n, b, x, w.r, st)) != CB_SUCCESS) return e;
                dot(w.r, w.r, n, w.partial, w.s, &w.s->rrn, st);
                if ((e = read_scal(w.s, h, st)) != CB_SUCCESS) return e;
                ++out.replacements;
                const double prev_anchor = anchor;
                anchor = std::sqrt(h.rrn);
                low = anchor;
                low_it = it;
                out.rel = rel_of(h, h.rrn);
                if (anchor <= target) {
                    out.converged = true;
                    return CB_SUCCESS;
                }
                // the low-precision products can no longer reduce the true residual
                if (anchor < 0.5 * best) {
                    best = anchor;
                    stalls = 0;
                } else if (++stalls >= 3) {
                    return CB_SUCCESS;
                }
                if (stalled || !(anchor < 0.5 * prev_anchor)) {
                    // restart: p = r; the next step's dot takes rr from the replaced rrn
                    ++out.restarts;
                    hipLaunchKernelGGL((copy_kernel<TV, TR>), dim3(g), dim3(kThreads), 0, st, w.p, w.r, n);
                    continue;
                }
            }
            if (h.bad) return CB_SUCCESS;  // not positive definite along a search direction
        }
        hipLaunchKernelGGL((update_p_kernel<TR, TV>), dim3(g), dim3(kThreads), 0, st, w.p, w.r, n, w.s);
    }
    return CB_SUCCESS;
}

// |b - A x| / |b| in FP64, the workspace's r as scratch
cb_status_t true_residual(cb_matrix_t A, int64_t n, const double *b, const double *x, const Work<double, double> &w,
                          hipStream_t st, double &rel, double &rr, double &bb) {
    cb_status_t e;
    hipLaunchKernelGGL(clear_scal_kernel, dim3(1), dim3(64), 0, st, w.s);
    if ((e = residual<double>(A, n, b, x, w.r, st)) != CB_SUCCESS) return e;
    dot(w.r, w.r, n, w.partial, w.s, &w.s->rr, st);
    dot(b, b, n, w.partial, w.s, &w.s->bb, st);
    Scal h{};
    if ((e = read_scal(w.s, h, st)) != CB_SUCCESS) return e;
    rr = h.rr;
    bb = h.bb;
    rel = rel_of(h, rr);
    return CB_SUCCESS;
}

cb_status_t check_opts(const cb_cg_options_t *opt, cb_cg_options_t &o) {
    cb_cg_options_default(&o);
    if (!opt) return CB_SUCCESS;
    if (opt->struct_size != sizeof(cb_cg_options_t)) return fail(CB_ERROR_INVALID_VALUE, "cb_cg_options_t.struct_size mismatch");
    o = *opt;
    if (o.max_iter < 1 || o.check_every < 1 || o.max_refine < 1 || !(o.rtol >= 0.0) || !(o.inner_rtol > 0.0) ||
        !(o.inner_rtol < 1.0) || !(o.replace_factor > 0.0) || !(o.replace_factor < 1.0) ||
        (o.refine_method != CB_REFINE_RESTART && o.refine_method != CB_REFINE_REPLACE))
        return fail(CB_ERROR_INVALID_VALUE, "invalid CG options");
    return CB_SUCCESS;
}

// restarted refinement (refine_method CB_REFINE_RESTART); TI: A_low's vector type
template <class TI>
cb_status_t refine_restart(cb_matrix_t A, cb_matrix_t A_low, int64_t n, const double *b, double *x, void *work,
                           const cb_cg_options_t &o, hipStream_t s, cb_cg_result_t &r) {
    const int g = blocks_for(n);
    constexpr int kI = (int)sizeof(TI);
    cb_status_t st;
    uint8_t *wb = static_cast<uint8_t *>(work);
    const Work<double, double> w64 = carve<double, double>(wb, n);
    const Work<TI, TI> wi = carve<TI, TI>(wb + cg_bytes(n, 8, 8), n);
    TI *rhs = reinterpret_cast<TI *>(wb + cg_bytes(n, 8, 8) + cg_bytes(n, kI, kI));
    TI *dsol = reinterpret_cast<TI *>(wb + cg_bytes(n, 8, 8) + cg_bytes(n, kI, kI) + align256((size_t)n * kI));
    double rel = 0.0, rr = 0.0, bb = 0.0;
    if ((st = true_residual(A, n, b, x, w64, s, rel, rr, bb)) != CB_SUCCESS) return st;
    int total = 0, outer = 0;
    const double target = o.rtol * std::sqrt(bb);
    while (std::sqrt(rr) > target && outer < o.max_refine) {
        // inner solve on r / |r| from d = 0
        hipLaunchKernelGGL(scale_to_kernel<TI>, dim3(g), dim3(kThreads), 0, s, rhs, w64.r, n, &w64.s->rr);
        hipLaunchKernelGGL(fill_kernel<TI>, dim3(g), dim3(kThreads), 0, s, dsol, n, TI(0));
        if ((st = hipcheck(hipGetLastError(), "refinement launch")) != CB_SUCCESS) return st;
        RunOut in;
        if ((st = cg_run<TI, TI>(A_low, nullptr, n, rhs, dsol, wi, o.inner_rtol, o.max_iter, o.check_every, 0.5, s,
                                 in)) != CB_SUCCESS)
            return st;
        total += in.iters;
        ++outer;
        hipLaunchKernelGGL(add_scaled_kernel<TI>, dim3(g), dim3(kThreads), 0, s, x, dsol, n, &w64.s->rr);
        if ((st = hipcheck(hipGetLastError(), "refinement launch")) != CB_SUCCESS) return st;
        const double prev = rr;
        if ((st = true_residual(A, n, b, x, w64, s, rel, rr, bb)) != CB_SUCCESS) return st;
        if (!(rr < prev)) break;  // no progress: the low-precision solve cannot reduce the residual further
    }
    r.converged = std::sqrt(rr) <= target;
    r.iterations = total;
    r.refinements = outer;
    r.rel_residual = rel;
    return CB_SUCCESS;
}

// Device addresses of the scratch array, per device, taken once with that device current; the mutex
// of a device also serialises the cb_cg_noalloc calls that share its array.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];
void *g_scratch[kMaxDevices];

// *ptr = this device's scratch address (looked up on the first call); the caller holds g_scratch_mu[dev]
cb_status_t scratch_address(int dev, void **ptr) {
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CB_ERROR_HIP, std::string("hipGetSymbolAddress of the solver scratch: ") + hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *ptr = g_scratch[dev];
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
    opt->refine_method = CB_REFINE_REPLACE;
    opt->replace_factor = 1e-2;
    return CB_SUCCESS;
}

cb_status_t cb_cg_workspace_bytes(cb_matrix_t A, cb_matrix_t A_low, int64_t *bytes) {
    if (!bytes) return fail(CB_ERROR_INVALID_VALUE, "NULL output");
    Mat M;
    cb_status_t st = mat_of(A, M);
    if (st != CB_SUCCESS) return st;
    size_t b = cg_bytes(M.n, M.esize, M.esize);
    if (A_low) {
        Mat L;
        if ((st = mat_of(A_low, L)) != CB_SUCCESS) return st;
        if (L.n != M.n) return fail(CB_ERROR_INVALID_VALUE, "the two matrices differ in size");
        b = refine_bytes(M.n, L.esize);
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
    if (work_bytes < (int64_t)cg_bytes(M.n, M.esize, M.esize)) return fail(CB_ERROR_INVALID_VALUE, "workspace too small");
    cb_cg_result_t r{};
    hipStream_t s = (hipStream_t)stream;
    if (M.n > 0) {
        RunOut out;
        if (M.esize == 8)
            st = cg_run<double, double>(A, nullptr, M.n, (const double *)b, (double *)x,
                                        carve<double, double>(work, M.n), o.rtol, o.max_iter, o.check_every, 0.5, s,
                                        out);
        else
            st = cg_run<float, float>(A, nullptr, M.n, (const float *)b, (float *)x, carve<float, float>(work, M.n),
                                      o.rtol, o.max_iter, o.check_every, 0.5, s, out);
        if (st != CB_SUCCESS) return st;
        r.converged = out.converged;
        r.iterations = out.iters;
        r.rel_residual = out.rel;
        if (M.esize == 8) {
            // report the true residual of the returned x (the recurrence drifts from it)
            double rel = 0.0, rr = 0.0, bb = 0.0;
            if ((st = true_residual(A, M.n, (const double *)b, (const double *)x, carve<double, double>(work, M.n), s,
                                    rel, rr, bb)) != CB_SUCCESS)
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
    if (work_bytes < (int64_t)refine_bytes(M.n, L.esize)) return fail(CB_ERROR_INVALID_VALUE, "workspace too small");
    cb_cg_result_t r{};
    if (M.n == 0) {
        r.converged = 1;
        *res = r;
        return CB_SUCCESS;
    }
    hipStream_t s = (hipStream_t)stream;
    if (o.refine_method == CB_REFINE_RESTART) {
        st = L.esize == 8 ? refine_restart<double>(A, A_low, M.n, b, x, work, o, s, r)
                          : refine_restart<float>(A, A_low, M.n, b, x, work, o, s, r);
        if (st != CB_SUCCESS) return st;
    } else {
        RunOut out;
        if (L.esize == 8)
            st = cg_run<double, double>(A_low, A, M.n, b, x, carve<double, double>(work, M.n), o.rtol, o.max_iter,
                                        o.check_every, o.replace_factor, s, out);
        else
            st = cg_run<double, float>(A_low, A, M.n, b, x, carve<double, float>(work, M.n), o.rtol, o.max_iter,
                                       o.check_every, o.replace_factor, s, out);
        if (st != CB_SUCCESS) return st;
        r.converged = out.converged;
        r.iterations = out.iters;
        r.refinements = out.replacements;
        r.restarts = out.restarts;
        r.rel_residual = out.rel;
        if (!out.converged) {
            // the held residual may be the recurrence's: report the true one
            double rel = 0.0, rr = 0.0, bb = 0.0;
            if ((st = true_residual(A, M.n, b, x, carve<double, double>(work, M.n), s, rel, rr, bb)) != CB_SUCCESS)
                return st;
            r.rel_residual = rel;
        }
    }
    *res = r;
    return CB_SUCCESS;
}

cb_status_t cb_cg_noalloc(cb_matrix_t A, const void *b, void *x, const cb_cg_options_t *opt, cb_cg_result_t *res,
                          void *stream) {
    Mat M;
    cb_status_t st = mat_of(A, M);
    if (st != CB_SUCCESS) return st;
    const int64_t need = (int64_t)cg_bytes(M.n, M.esize, M.esize);
    if (need > (int64_t)CB_CG_NOALLOC_MAX_BYTES)
        return fail(CB_ERROR_INVALID_VALUE, "cb_cg_noalloc: the solve needs " + std::to_string(need) +
                                                " bytes of workspace, more than its fixed " +
                                                std::to_string((int64_t)CB_CG_NOALLOC_MAX_BYTES) +
                                                " (use cb_cg with a caller workspace)");
    cbh::MatrixView v;
    if ((st = cbh::matrix_view(A, v)) != CB_SUCCESS) return st;
    int dev = -1;
    if ((st = hipcheck(hipGetDevice(&dev), "hipGetDevice")) != CB_SUCCESS) return st;
    if (dev != v.device) return fail(CB_ERROR_INVALID_VALUE, "cb_cg_noalloc: the matrix lives on another device than the current one");
    if (dev < 0 || dev >= kMaxDevices) return fail(CB_ERROR_NOT_SUPPORTED, "cb_cg_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
    void *work = nullptr;
    if ((st = scratch_address(dev, &work)) != CB_SUCCESS) return st;
    st = cb_cg(A, b, x, work, need, opt, res, stream);
    // the array is free for the next call only once this solve's kernels have finished
    const cb_status_t sync = hipcheck(hipStreamSynchronize((hipStream_t)stream), "stream synchronize");
    return st != CB_SUCCESS ? st : sync;
}

}  // extern "C"
