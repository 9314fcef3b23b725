// Serving loop: resident matrices, continuous batching of SpMM requests and CG solves.
//
// One worker thread per server owns every HIP call.  Requests wait in arrival order and are
// admitted when their vectors fit in the server's arena (one device allocation made at creation,
// handed out first-fit) and, for a solve, a solve slot of its vector type is free.  The active
// solves advance together in periods of check_every steps; a step is the products of all of them
// (one batched launch per value type, aggregation and row-sum mode, covering the work ranges of
// all their matrices) followed by batched vector updates with one grid row per solve.  A period
// is captured once as a HIP graph and replayed until the active set changes.  After each period
// the solves' scalars come back to the host, finished solves return their x and leave, and queued
// solves join.  SpMM requests run on streams of their own beside the periods.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cb_host.h"
#include "cb_internal.h"
#include "cbspmv.h"

namespace {

constexpr int kT = 256;   // threads per block of the solve kernels
constexpr int kGB = 64;   // blocks per solve in the batched vector kernels (the reduction order)
constexpr size_t kAlign = 256;
constexpr size_t kMaxMatrices = 1 << 14;  // registered handles (storage reserved up front, so the
                                          // worker reads entries while new ones are appended)

using Clock = std::chrono::steady_clock;

struct SolveScal {
    double rr, pq, rrn, bb;
    double rr0;  // r.r at the solve's start (or its last residual replacement)
    int32_t bad, pad;
};

// one active solve: x, r, b in TX; the direction p and the product q = A p in TP, the vector type
// of the matrix the steps multiply by (TP = TX for plain CG; float with TX = double for a refined
// solve, whose products run on a FP32/BF16 copy)
template <class TX, class TP>
struct SolveJob {
    TX *x, *r;
    TP *p, *q;
    const TX *b;
    int64_t n;
    int32_t active;
    int32_t zero_q;  // the product's shared or empty panels need q cleared before it
};

__device__ double block_sum(double v) {
    __shared__ double sh[kT / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kT / 64; ++i) s += sh[i];
    return s;
}

// grid (kGB, solves): block sums of p.q per solve
template <class TX, class TP>
__global__ __launch_bounds__(kT) void sb_dot_pq(const SolveJob<TX, TP> *__restrict__ jobs, double *__restrict__ partial) {
    const SolveJob<TX, TP> &J = jobs[blockIdx.y];
    if (!J.active) return;
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < J.n; i += (int64_t)kGB * kT)
        v += (double)J.p[i] * (double)J.q[i];
    const double s = block_sum(v);
    if (threadIdx.x == 0) partial[blockIdx.y * kGB + blockIdx.x] = s;
}

static_assert(kGB == 64, "one block sum per lane of the reduction");

// the kGB block sums of one solve added as sb_reduce adds them (one per lane of the first
// wavefront, then a shuffle tree), so every block of a kernel sees the same value
__device__ double solve_total(const double *__restrict__ part) {
    __shared__ double tot;
    if (threadIdx.x < 64) {
        double v = part[threadIdx.x];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
        if (threadIdx.x == 0) tot = v;
    }
    __syncthreads();
    return tot;
}

// grid (solves), 64 threads: the kGB block sums of a solve in block order; mode 2 (one solve, its
// start): rr = rrn = sum; mode 3 (one solve): bb = sum, pq = 0, bad = 0.  (The steps add their block
// sums inside the kernels that use them, solve_total.)
template <class TX, class TP>
__global__ __launch_bounds__(64) void sb_reduce(const SolveJob<TX, TP> *__restrict__ jobs, const double *__restrict__ partial,
                                                SolveScal *__restrict__ scal, int mode, int one) {
    const int j = one >= 0 ? one : (int)blockIdx.x;
    if (!jobs[j].active) return;
    double v = partial[j * kGB + threadIdx.x];  // kGB == 64: one block sum per lane
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if (threadIdx.x == 0) {
        SolveScal &s = scal[j];
        if (mode == 2) {
            s.rr = v;
            s.rrn = v;
            s.rr0 = v;
        } else {
            s.bb = v;
            s.pq = 0.0;
            s.bad = 0;
        }
    }
}

// grid (kGB, solves): x += alpha p, r -= alpha q with alpha = rr / pq, where pq adds the block sums
// of p.q (pq_part) and rr is the previous step's new r.r (rrn); block sums of the new r.r (rr_part).
// Block 0 records rr and pq for sb_update_p and the host; no other block reads them here.
template <class TX, class TP>
__global__ __launch_bounds__(kT) void sb_update_xr(const SolveJob<TX, TP> *__restrict__ jobs, SolveScal *__restrict__ scal,
                                                   const double *__restrict__ pq_part, double *__restrict__ rr_part) {
    const SolveJob<TX, TP> &J = jobs[blockIdx.y];
    if (!J.active) return;
    SolveScal &s = scal[blockIdx.y];
    const double pq = solve_total(pq_part + blockIdx.y * kGB);
    const double rr = s.rrn;
    const bool ok = pq > 0.0 && std::isfinite(pq);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s.rr = rr;
        s.pq = pq;
        if (!ok) s.bad = 1;
    }
    const double alpha = ok ? rr / pq : 0.0;
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < J.n; i += (int64_t)kGB * kT) {
        J.x[i] = (TX)((double)J.x[i] + alpha * (double)J.p[i]);
        const TX ri = (TX)((double)J.r[i] - alpha * (double)J.q[i]);
        J.r[i] = ri;
        v += (double)ri * (double)ri;
    }
    const double sum = block_sum(v);
    if (threadIdx.x == 0) rr_part[blockIdx.y * kGB + blockIdx.x] = sum;
}

// grid (kGB, solves): p = r + beta p with beta = rrn / rr, where rrn adds the block sums of the new
// r.r (rr_part); q cleared where the product needs it.  Block 0 records rrn for the next step and
// the host; no other block reads it here.
template <class TX, class TP>
__global__ __launch_bounds__(kT) void sb_update_p(const SolveJob<TX, TP> *__restrict__ jobs, SolveScal *__restrict__ scal,
                                                  const double *__restrict__ rr_part) {
    const SolveJob<TX, TP> &J = jobs[blockIdx.y];
    if (!J.active) return;
    SolveScal &s = scal[blockIdx.y];
    const double rrn = solve_total(rr_part + blockIdx.y * kGB);
    const double rr = s.rr;
    if (blockIdx.x == 0 && threadIdx.x == 0) s.rrn = rrn;
    const double beta = rr > 0.0 ? rrn / rr : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < J.n; i += (int64_t)kGB * kT) {
        J.p[i] = (TP)((double)J.r[i] + beta * (double)J.p[i]);
        if (J.zero_q) J.q[i] = TP(0);
    }
}

// one solve's start: r = b (before r -= A x), then p = r and q = 0; block sums of a.b
template <class T>
__global__ __launch_bounds__(kT) void sb_copy(T *__restrict__ dst, const T *__restrict__ src, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) dst[i] = src[i];
}
template <class TX, class TP>
__global__ __launch_bounds__(kT) void sb_start(TP *__restrict__ p, TP *__restrict__ q, const TX *__restrict__ r,
                                               int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        p[i] = (TP)r[i];
        q[i] = TP(0);
    }
}
// a refined solve's residual replacement, second half: t holds the true residual b - A x (FP64
// matrix); r takes its place, and the direction either restarts (p = t) or keeps its Krylov
// history with the residual part corrected (p += t - r, so p = t + beta p_old as if the step's p
// update had used the true residual)
__global__ __launch_bounds__(kT) void sb_replace(float *__restrict__ p, double *__restrict__ r,
                                                 const double *__restrict__ t, int64_t n, int restart) {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        const double ti = t[i];
        p[i] = restart ? (float)ti : (float)((double)p[i] + (ti - r[i]));
        r[i] = ti;
    }
}
template <class T>
__global__ __launch_bounds__(kT) void sb_dot_one(const T *__restrict__ a, const T *__restrict__ b, int64_t n,
                                                 double *__restrict__ partial) {
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)kGB * kT)
        v += (double)a[i] * (double)b[i];
    const double s = block_sum(v);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// first-fit allocator over [0, size)
class Arena {
  public:
    void init(size_t size) {
        size_ = size;
        free_.clear();
        if (size) free_[0] = size;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t &off) {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes ? bytes : 1);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t peak() const { return peak_; }

  private:
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Req {
    int64_t ticket = 0;
    cb_request_t r{};
    Clock::time_point t_submit, t_admit;
    size_t off = 0, bytes = 0;
    int slot = -1;     // solve slot
    int stream = -1;   // SpMM stream
    hipEvent_t ev = nullptr;
    int iters = 0;
    int max_iter = 500;
    double rtol = 1e-10;
    int conv = 0;      // outcome of a finished solve, reported once its x has landed
    double rel = 0.0;
    bool failed = false;
    int pm = -1;       // the matrix the solve's steps multiply by (matrix_low for a refined solve)
    // refined solves: the true residual's device vector and the replacement state (as cb_cg_refine)
    double *t = nullptr;
    const double *b64 = nullptr;
    double *x64 = nullptr;
    double anchor = 0.0, best = 0.0, low = 0.0;
    int low_it = 0, stalls = 0, repl = 0, restarts = 0;
};

struct Mat {
    cb_matrix_t A;
    cbh::MatrixView v;
    int esize;  // vector element bytes
};

// solve slots and device tables of one pair of vector types (solution and residual TX, direction
// and product TP)
template <class TX, class TP>
struct Group {
    int S = 0;
    std::vector<SolveJob<TX, TP>> jobs;  // host copy of the table
    std::vector<Req *> req;              // slot -> request
    SolveJob<TX, TP> *d_jobs = nullptr;
    SolveScal *d_scal = nullptr;
    double *d_partial = nullptr;
    SolveScal *h_scal = nullptr;  // pinned
    int active = 0;
    int top = 0;  // slots [0, top) hold every active solve
    // batched products: per (kernel value code, aggregation, row-sum mode)
    struct Launch {
        int kvt, agg, rr, quad, lt, first, count, total;
    };
    std::vector<Launch> launches;
    cbd::BatchJob *d_bjobs = nullptr;
    int32_t *d_wave_job = nullptr;
    size_t wave_cap = 0;
};

}  // namespace

struct cb_server_s {
    cb_server_options_t o{};
    int device = 0;
    void *arena_base = nullptr;
    Arena arena;
    std::vector<Mat> mats;
    Group<double, double> g64;
    Group<float, float> g32;
    Group<double, float> gmx;  // refined solves: FP64 x and r, float p and q on a FP32/BF16 copy
    hipStream_t cg_stream = nullptr;
    std::vector<hipStream_t> spmm_streams;
    hipEvent_t period_ev = nullptr;
    hipGraphExec_t graph = nullptr;
    bool dirty = true;
    int same_periods = 0;  // periods run since the active set last changed
    bool period_inflight = false;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    // a list: the worker walks it with the lock released around each admission while submit()
    // appends, and list insertions leave the worker's iterator valid (a deque's would not be)
    std::list<Req *> pending;
    std::list<Req *> spmm_inflight;
    std::unordered_map<int64_t, cb_response_t> resp;
    int64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;

    // statistics (guarded by mu)
    std::vector<double> lat_us;
    int64_t submitted = 0, rejected = 0, spmm_done = 0, cg_done = 0, steps = 0;
    int active_peak = 0, graph_builds = 0;
    bool started = false;
    Clock::time_point t_first, t_last;

    void run();
    bool admit_one(Req *q, bool &blocked_by_memory);
    template <class TX, class TP>
    int start_solve(Group<TX, TP> &g, Req *q, const Mat &Mh, const Mat &Ml);
    template <class TX, class TP>
    void retire_solves(Group<TX, TP> &g, std::vector<Req *> &done);
    void retire_refined(std::vector<Req *> &done);
    template <class TX, class TP>
    hipError_t build_launches(Group<TX, TP> &g);
    template <class TX, class TP>
    hipError_t enqueue_steps(Group<TX, TP> &g, int nsteps);
    hipError_t enqueue_period();
    void complete(Req *q, cb_status_t st, int iters, int conv, double rel);
};

namespace {

cb_status_t fail(cb_status_t st, const std::string &msg) {
    cbh::set_last_error(msg);
    return st;
}

cb_status_t hipfail(hipError_t e, const char *what) {
    return fail(CB_ERROR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class TX, class TP>
hipError_t group_alloc(Group<TX, TP> &g, int S) {
    g.S = S;
    g.jobs.assign(S, SolveJob<TX, TP>{});
    g.req.assign(S, nullptr);
    hipError_t e;
    if ((e = hipMalloc(&g.d_jobs, sizeof(SolveJob<TX, TP>) * S)) != hipSuccess) return e;
    if ((e = hipMalloc(&g.d_scal, sizeof(SolveScal) * S)) != hipSuccess) return e;
    // two sets of block sums: p.q (written by sb_dot_pq, read by sb_update_xr) and r.r (written by
    // sb_update_xr, read by sb_update_p), so no kernel reads the set it writes
    if ((e = hipMalloc(&g.d_partial, sizeof(double) * kGB * 2 * S)) != hipSuccess) return e;
    if ((e = hipMalloc(&g.d_bjobs, sizeof(cbd::BatchJob) * S)) != hipSuccess) return e;
    if ((e = hipHostMalloc(&g.h_scal, sizeof(SolveScal) * S, hipHostMallocDefault)) != hipSuccess) return e;
    return hipMemcpy(g.d_jobs, g.jobs.data(), sizeof(SolveJob<TX, TP>) * S, hipMemcpyHostToDevice);
}

template <class TX, class TP>
void group_free(Group<TX, TP> &g) {
    hipFree(g.d_jobs);
    hipFree(g.d_scal);
    hipFree(g.d_partial);
    hipFree(g.d_bjobs);
    hipFree(g.d_wave_job);
    if (g.h_scal) hipHostFree(g.h_scal);
}

double us_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::micro>(b - a).count();
}

}  // namespace

// arena bytes of a request
static size_t footprint(const cb_request_t &r, const Mat &M) {
    const size_t es = (size_t)M.esize;
    if (r.kind == CB_REQ_SPMM)
        return align_up((size_t)M.v.n * r.k * es) + align_up((size_t)M.v.m * r.k * es);
    if (r.kind == CB_REQ_CG_REFINE)  // b, x, r, t in FP64, p, q in float
        return 4 * align_up((size_t)M.v.n * sizeof(double)) + 2 * align_up((size_t)M.v.n * sizeof(float));
    return 5 * align_up((size_t)M.v.n * es);  // b, x, r, p, q
}

void cb_server_s::complete(Req *q, cb_status_t st, int iters, int conv, double rel) {
    const auto now = Clock::now();
    cb_response_t rs{};
    rs.done = 1;
    rs.status = st;
    rs.iterations = iters;
    rs.converged = conv;
    rs.rel_residual = rel;
    rs.latency_us = us_between(q->t_submit, now);
    rs.queue_us = us_between(q->t_submit, q->t_admit);
    rs.replacements = q->repl;
    rs.restarts = q->restarts;
    {
        std::lock_guard<std::mutex> lk(mu);
        resp[q->ticket] = rs;
        lat_us.push_back(rs.latency_us);
        if (q->r.kind == CB_REQ_SPMM) ++spmm_done;
        else ++cg_done;
        t_last = now;
    }
    cv_done.notify_all();
    if (q->bytes) arena.release(q->off, q->bytes);
    if (q->ev) hipEventDestroy(q->ev);
    delete q;
}

// 1: the solve started; 0: no free slot; -1: a HIP call failed (nothing is left in the slot).
// Mh: the system's matrix (r = b - Mh x at the start); Ml: the matrix the steps multiply by (Mh
// itself for plain CG, its FP32/BF16 copy for a refined solve)
template <class TX, class TP>
int cb_server_s::start_solve(Group<TX, TP> &g, Req *q, const Mat &Mh, const Mat &Ml) {
    int slot = -1;
    for (int i = 0; i < g.S; ++i)
        if (!g.req[i]) {
            slot = i;
            break;
        }
    if (slot < 0) return 0;
    const int64_t n = Mh.v.n;
    const size_t vb = align_up((size_t)n * sizeof(TX)), vp = align_up((size_t)n * sizeof(TP));
    uint8_t *base = static_cast<uint8_t *>(arena_base) + q->off;
    TX *b = reinterpret_cast<TX *>(base), *x = reinterpret_cast<TX *>(base + vb), *r = reinterpret_cast<TX *>(base + 2 * vb);
    TP *p = reinterpret_cast<TP *>(base + 3 * vb), *qq = reinterpret_cast<TP *>(base + 3 * vb + vp);
    if (q->r.kind == CB_REQ_CG_REFINE) {
        q->t = reinterpret_cast<double *>(base + 3 * vb + 2 * vp);
        q->b64 = reinterpret_cast<const double *>(b);
        q->x64 = reinterpret_cast<double *>(x);
    }
    hipStream_t s = cg_stream;
    hipError_t e = hipSuccess;
    if (n > 0) {
        e = hipMemcpyAsync(b, q->r.in, n * sizeof(TX), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(x, q->r.out, n * sizeof(TX), hipMemcpyHostToDevice, s);
        const int gb = (int)std::min<int64_t>(1024, (n + kT - 1) / kT);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(sb_copy<TX>, dim3(gb), dim3(kT), 0, s, r, b, n);
            e = hipGetLastError();
        }
        if (e == hipSuccess && cb_spmv(Mh.A, -1.0, x, 1.0, r, s) != CB_SUCCESS) e = hipErrorLaunchFailure;  // r = b - A x
        if (e == hipSuccess) {
            hipLaunchKernelGGL((sb_start<TX, TP>), dim3(gb), dim3(kT), 0, s, p, qq, r, n);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) return -1;
    SolveJob<TX, TP> J{};
    J.x = x;
    J.r = r;
    J.p = p;
    J.q = qq;
    J.b = b;
    J.n = n;
    J.active = 1;
    J.zero_q = Ml.v.nprepass > 0;
    g.jobs[slot] = J;
    g.req[slot] = q;
    q->slot = slot;
    e = hipMemcpyAsync(g.d_jobs + slot, &g.jobs[slot], sizeof(SolveJob<TX, TP>), hipMemcpyHostToDevice, s);
    double *part = g.d_partial + (size_t)slot * kGB;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(sb_dot_one<TX>, dim3(kGB), dim3(kT), 0, s, r, r, n, part);
        hipLaunchKernelGGL((sb_reduce<TX, TP>), dim3(1), dim3(64), 0, s, g.d_jobs, g.d_partial, g.d_scal, 2, slot);
        hipLaunchKernelGGL(sb_dot_one<TX>, dim3(kGB), dim3(kT), 0, s, b, b, n, part);
        hipLaunchKernelGGL((sb_reduce<TX, TP>), dim3(1), dim3(64), 0, s, g.d_jobs, g.d_partial, g.d_scal, 3, slot);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        g.jobs[slot].active = 0;
        g.req[slot] = nullptr;
        q->slot = -1;
        return -1;
    }
    // the host copy of the table must outlive the copy above: it is only rewritten between periods
    ++g.active;
    g.top = std::max(g.top, slot + 1);
    dirty = true;
    return 1;
}

bool cb_server_s::admit_one(Req *q, bool &blocked_by_memory) {
    blocked_by_memory = false;
    const Mat &M = mats[q->r.matrix];
    if (q->r.kind == CB_REQ_CG) {
        if (period_inflight) return false;
        if ((M.esize == 8 && g64.active >= g64.S) || (M.esize == 4 && g32.active >= g32.S)) return false;
    } else if (q->r.kind == CB_REQ_CG_REFINE) {
        if (period_inflight || gmx.active >= gmx.S) return false;
    }
    size_t off = 0;
    const size_t bytes = footprint(q->r, M);
    if (!arena.alloc(bytes, off)) {
        blocked_by_memory = true;
        return false;
    }
    q->off = off;
    q->bytes = bytes;
    q->t_admit = Clock::now();
    if (q->r.kind == CB_REQ_CG || q->r.kind == CB_REQ_CG_REFINE) {
        const int ok = q->r.kind == CB_REQ_CG_REFINE ? start_solve(gmx, q, M, mats[q->pm])
                       : M.esize == 8                ? start_solve(g64, q, M, M)
                                                     : start_solve(g32, q, M, M);
        if (ok == 0) {
            arena.release(off, bytes);
            q->bytes = 0;
            return false;
        }
        if (ok < 0) {
            hipStreamSynchronize(cg_stream);
            hipGetLastError();
            complete(q, CB_ERROR_HIP, 0, 0, 0.0);
        }
        return true;
    }
    // SpMM on the least recently used stream
    const int si = (int)(q->ticket % (int64_t)spmm_streams.size());
    hipStream_t s = spmm_streams[si];
    const size_t es = (size_t)M.esize;
    uint8_t *base = static_cast<uint8_t *>(arena_base) + off;
    void *X = base, *Y = base + align_up((size_t)M.v.n * q->r.k * es);
    const size_t xb = (size_t)M.v.n * q->r.k * es, yb = (size_t)M.v.m * q->r.k * es;
    cb_status_t st = CB_SUCCESS;
    hipError_t e = hipSuccess;
    if (xb) e = hipMemcpyAsync(X, q->r.in, xb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && yb && q->r.beta != 0.0) e = hipMemcpyAsync(Y, q->r.out, yb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) st = cb_spmm(M.A, q->r.k, q->r.alpha, X, q->r.k, q->r.beta, Y, q->r.k, s);
    if (e == hipSuccess && st == CB_SUCCESS && yb) e = hipMemcpyAsync(q->r.out, Y, yb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && st == CB_SUCCESS) e = hipEventCreateWithFlags(&q->ev, hipEventDisableTiming);
    if (e == hipSuccess && st == CB_SUCCESS) e = hipEventRecord(q->ev, s);
    q->stream = si;
    if (e != hipSuccess || st != CB_SUCCESS) {
        hipStreamSynchronize(s);
        hipGetLastError();
        complete(q, st != CB_SUCCESS ? st : CB_ERROR_HIP, 0, 0, 0.0);
        return true;
    }
    spmm_inflight.push_back(q);
    return true;
}

template <class TX, class TP>
hipError_t cb_server_s::build_launches(Group<TX, TP> &g) {
    g.launches.clear();
    if (!g.active) return hipSuccess;
    // order the active solves by (kernel value code, tile size, batch format, aggregation, row-sum mode)
    std::vector<int> order;
    for (int i = 0; i < g.top; ++i)
        if (g.req[i]) order.push_back(i);
    auto key = [&](int i) {
        const cbh::MatrixView &v = mats[g.req[i]->pm].v;
        return v.kernel_vt * 128 + (v.view.tile_lt == 3 ? 64 : 0) + (v.view.spmv_kernel == 2 ? 32 : 0) +
               v.col_agg * 8 + v.row_reduce;  // row_reduce < 8, col_agg < 4
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
    std::vector<cbd::BatchJob> bj;
    std::vector<int32_t> wave_job;
    size_t i = 0;
    while (i < order.size()) {
        const int k0 = key(order[i]);
        typename Group<TX, TP>::Launch L{};
        const cbh::MatrixView &v0 = mats[g.req[order[i]]->pm].v;
        L.kvt = v0.kernel_vt;
        L.agg = v0.col_agg;
        L.rr = v0.row_reduce;
        L.quad = v0.view.spmv_kernel == 2 ? 1 : 0;
        L.lt = v0.view.tile_lt;
        L.first = (int)bj.size();
        L.total = 0;
        for (; i < order.size() && key(order[i]) == k0; ++i) {
            const int slot = order[i];
            const cbh::MatrixView &v = mats[g.req[slot]->pm].v;
            cbd::BatchJob J{};
            J.d = v.view;
            J.x = g.jobs[slot].p;
            J.y = g.jobs[slot].q;
            J.alpha = 1.0;
            J.beta = 0.0;
            J.wave_base = L.total;
            const int jid = (int)bj.size() - L.first;
            for (int w = 0; w < v.view.nwaves; ++w) wave_job.push_back(jid);
            L.total += v.view.nwaves;
            bj.push_back(J);
        }
        L.count = (int)bj.size() - L.first;
        g.launches.push_back(L);
    }
    hipError_t e;
    if (wave_job.size() > g.wave_cap) {
        if (g.d_wave_job) hipFree(g.d_wave_job);
        g.wave_cap = std::max<size_t>(wave_job.size(), 2 * g.wave_cap);
        if ((e = hipMalloc(&g.d_wave_job, sizeof(int32_t) * g.wave_cap)) != hipSuccess) return e;
    }
    if ((e = hipMemcpy(g.d_bjobs, bj.data(), sizeof(cbd::BatchJob) * bj.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    // wave_job: each launch's slice numbers its jobs from the launch's first
    if (!wave_job.empty())
        if ((e = hipMemcpy(g.d_wave_job, wave_job.data(), sizeof(int32_t) * wave_job.size(), hipMemcpyHostToDevice)) !=
            hipSuccess)
            return e;
    return hipMemcpy(g.d_jobs, g.jobs.data(), sizeof(SolveJob<TX, TP>) * g.S, hipMemcpyHostToDevice);
}

template <class TX, class TP>
hipError_t cb_server_s::enqueue_steps(Group<TX, TP> &g, int nsteps) {
    if (!g.active) return hipSuccess;
    hipStream_t s = cg_stream;
    const dim3 grid(kGB, g.top);
    for (int step = 0; step < nsteps; ++step) {
        size_t wofs = 0;
        for (const auto &L : g.launches) {
            hipError_t e = cbd::launch_spmv_batch(g.d_bjobs + L.first, g.d_wave_job + wofs, L.total, L.kvt, L.agg, L.rr,
                                                   L.quad, L.lt, s);
            if (e != hipSuccess) return e;
            wofs += (size_t)L.total;
        }
        double *pq_part = g.d_partial, *rr_part = g.d_partial + (size_t)kGB * g.S;
        hipLaunchKernelGGL((sb_dot_pq<TX, TP>), grid, dim3(kT), 0, s, g.d_jobs, pq_part);
        hipLaunchKernelGGL((sb_update_xr<TX, TP>), grid, dim3(kT), 0, s, g.d_jobs, g.d_scal, pq_part, rr_part);
        hipLaunchKernelGGL((sb_update_p<TX, TP>), grid, dim3(kT), 0, s, g.d_jobs, g.d_scal, rr_part);
    }
    return hipGetLastError();
}

hipError_t cb_server_s::enqueue_period() {
    hipError_t e;
    if (dirty) {
        if ((e = build_launches(g64)) != hipSuccess) return e;
        if ((e = build_launches(g32)) != hipSuccess) return e;
        if ((e = build_launches(gmx)) != hipSuccess) return e;
        if (graph) {
            hipGraphExecDestroy(graph);
            graph = nullptr;
        }
        dirty = false;
        same_periods = 0;
    }
    // the first period of a new active set runs as plain launches: under steady arrivals most sets
    // last one period, and capturing a graph for one replay costs more than it saves; from the
    // second period on the set is captured once and replayed
    const bool replay = o.use_graph && same_periods >= 1;
    ++same_periods;
    if (replay && !graph) {
        hipGraph_t gr = nullptr;
        if ((e = hipStreamBeginCapture(cg_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
        hipError_t e1 = enqueue_steps(g64, o.check_every);
        hipError_t e2 = enqueue_steps(g32, o.check_every);
        hipError_t e3 = enqueue_steps(gmx, o.check_every);
        e = hipStreamEndCapture(cg_stream, &gr);
        if (e1 != hipSuccess) return e1;
        if (e2 != hipSuccess) return e2;
        if (e3 != hipSuccess) return e3;
        if (e != hipSuccess) return e;
        e = hipGraphInstantiate(&graph, gr, nullptr, nullptr, 0);
        hipGraphDestroy(gr);
        if (e != hipSuccess) return e;
        std::lock_guard<std::mutex> lk(mu);
        ++graph_builds;
    }
    if (replay) {
        if ((e = hipGraphLaunch(graph, cg_stream)) != hipSuccess) return e;
    } else {
        if ((e = enqueue_steps(g64, o.check_every)) != hipSuccess) return e;
        if ((e = enqueue_steps(g32, o.check_every)) != hipSuccess) return e;
        if ((e = enqueue_steps(gmx, o.check_every)) != hipSuccess) return e;
    }
    if (g64.active)
        hipMemcpyAsync(g64.h_scal, g64.d_scal, sizeof(SolveScal) * g64.top, hipMemcpyDeviceToHost, cg_stream);
    if (g32.active)
        hipMemcpyAsync(g32.h_scal, g32.d_scal, sizeof(SolveScal) * g32.top, hipMemcpyDeviceToHost, cg_stream);
    if (gmx.active)
        hipMemcpyAsync(gmx.h_scal, gmx.d_scal, sizeof(SolveScal) * gmx.top, hipMemcpyDeviceToHost, cg_stream);
    return hipEventRecord(period_ev, cg_stream);
}

template <class TX, class TP>
void cb_server_s::retire_solves(Group<TX, TP> &g, std::vector<Req *> &done) {
    for (int i = 0; i < g.top; ++i) {
        Req *q = g.req[i];
        if (!q) continue;
        q->iters += o.check_every;
        const SolveScal &s = g.h_scal[i];
        const bool conv = std::sqrt(s.rrn) <= q->rtol * std::sqrt(s.bb);
        if (conv || s.bad || q->iters >= q->max_iter) {
            // x back to the caller
            if (hipMemcpyAsync(q->r.out, g.jobs[i].x, (size_t)g.jobs[i].n * sizeof(TX), hipMemcpyDeviceToHost,
                               cg_stream) != hipSuccess)
                q->failed = true;
            q->slot = -1;
            g.req[i] = nullptr;
            g.jobs[i].active = 0;
            --g.active;
            dirty = true;
            q->conv = conv ? 1 : 0;
            q->rel = s.bb > 0.0 ? std::sqrt(s.rrn / s.bb) : std::sqrt(s.rrn);
            done.push_back(q);
        }
    }
    while (g.top > 0 && !g.req[g.top - 1]) --g.top;
}

// End of a period for the refined solves (as cb_cg_refine's residual replacement): a solve whose
// recurrence residual has fallen by kReplaceFactor since its last replacement, reached the
// tolerance, made no new low (10 % below the last) for eight checks, or used its iterations has r
// replaced by the true FP64 residual b - A x; only a true residual ends a solve as converged.  The
// direction keeps its history unless the replacement came from a stall or the true residual has
// not halved since the previous one (restart, p = r); three replacements without halving the best
// true residual end the solve unconverged.  Replacements run between periods, with one wait for
// their norms.
constexpr double kReplaceFactor = 1e-2;

void cb_server_s::retire_refined(std::vector<Req *> &done) {
    Group<double, float> &g = gmx;
    if (!g.active) return;
    const int ce = o.check_every;
    auto finish = [&](int i, int conv, double rel) {
        Req *q = g.req[i];
        if (g.jobs[i].n > 0 &&
            hipMemcpyAsync(q->r.out, g.jobs[i].x, (size_t)g.jobs[i].n * sizeof(double), hipMemcpyDeviceToHost,
                           cg_stream) != hipSuccess)
            q->failed = true;
        q->slot = -1;
        g.req[i] = nullptr;
        g.jobs[i].active = 0;
        --g.active;
        dirty = true;
        q->conv = conv;
        q->rel = rel;
        done.push_back(q);
    };
    std::vector<int> repl;
    std::vector<char> stalled(g.top, 0);
    for (int i = 0; i < g.top; ++i) {
        Req *q = g.req[i];
        if (!q) continue;
        q->iters += ce;
        const SolveScal &s = g.h_scal[i];
        if (q->anchor < 0.0) q->anchor = q->best = q->low = std::sqrt(s.rr0);
        const double target = q->rtol * std::sqrt(s.bb), rn = std::sqrt(s.rrn);
        if (s.bad || !std::isfinite(rn)) {  // not positive definite along a direction, or overflow
            finish(i, 0, s.bb > 0.0 ? rn / std::sqrt(s.bb) : rn);
            continue;
        }
        if (rn < 0.9 * q->low) {
            q->low = rn;
            q->low_it = q->iters;
        }
        const bool stall = q->iters - q->low_it >= 8 * ce;
        if (rn <= target || rn <= kReplaceFactor * q->anchor || stall || q->iters >= q->max_iter) {
            stalled[i] = rn > target && rn > kReplaceFactor * q->anchor;
            repl.push_back(i);
        }
    }
    if (!repl.empty()) {
        // the true residuals t = b - A x with the FP64 matrix, their squares into rr0 (and rr, rrn)
        hipStream_t st = cg_stream;
        for (int i : repl) {
            Req *q = g.req[i];
            const int64_t n = g.jobs[i].n;
            if (n > 0) {
                const int gb = (int)std::min<int64_t>(1024, (n + kT - 1) / kT);
                hipLaunchKernelGGL(sb_copy<double>, dim3(gb), dim3(kT), 0, st, q->t, q->b64, n);
                if (cb_spmv(mats[q->r.matrix].A, -1.0, q->x64, 1.0, q->t, st) != CB_SUCCESS) q->failed = true;
            }
            hipLaunchKernelGGL(sb_dot_one<double>, dim3(kGB), dim3(kT), 0, st, q->t, q->t, n,
                               g.d_partial + (size_t)i * kGB);
            hipLaunchKernelGGL((sb_reduce<double, float>), dim3(1), dim3(64), 0, st, g.d_jobs, g.d_partial, g.d_scal, 2,
                               i);
        }
        if (hipMemcpyAsync(g.h_scal, g.d_scal, sizeof(SolveScal) * g.top, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            for (int i : repl) g.req[i]->failed = true;
        for (int i : repl) {
            Req *q = g.req[i];
            const SolveScal &s = g.h_scal[i];
            const double target = q->rtol * std::sqrt(s.bb), prev = q->anchor;
            ++q->repl;
            q->anchor = q->low = std::sqrt(s.rr0);
            q->low_it = q->iters;
            const double rel = s.bb > 0.0 ? q->anchor / std::sqrt(s.bb) : q->anchor;
            if (q->failed || q->anchor <= target || q->iters >= q->max_iter || !std::isfinite(q->anchor)) {
                finish(i, !q->failed && q->anchor <= target ? 1 : 0, rel);
                continue;
            }
            if (q->anchor < 0.5 * q->best) {
                q->best = q->anchor;
                q->stalls = 0;
            } else if (++q->stalls >= 3) {
                finish(i, 0, rel);
                continue;
            }
            const int restart = stalled[i] || !(q->anchor < 0.5 * prev) ? 1 : 0;
            q->restarts += restart;
            const int64_t n = g.jobs[i].n;
            if (n > 0) {
                const int gb = (int)std::min<int64_t>(1024, (n + kT - 1) / kT);
                hipLaunchKernelGGL(sb_replace, dim3(gb), dim3(kT), 0, st, g.jobs[i].p, g.jobs[i].r, q->t, n, restart);
            }
        }
    }
    while (g.top > 0 && !g.req[g.top - 1]) --g.top;
}

void cb_server_s::run() {
    hipSetDevice(device);
    for (;;) {
        bool progressed = false;
        // SpMM completions
        for (auto it = spmm_inflight.begin(); it != spmm_inflight.end();) {
            if (hipEventQuery((*it)->ev) == hipSuccess) {
                Req *q = *it;
                it = spmm_inflight.erase(it);
                complete(q, CB_SUCCESS, 0, 0, 0.0);
                progressed = true;
            } else {
                ++it;
            }
        }
        // end of a solve period: retire finished solves
        if (period_inflight && hipEventQuery(period_ev) == hipSuccess) {
            period_inflight = false;
            {
                std::lock_guard<std::mutex> lk(mu);
                steps += o.check_every;
            }
            std::vector<Req *> done;
            retire_solves(g64, done);
            retire_solves(g32, done);
            retire_refined(done);
            if (!done.empty()) hipStreamSynchronize(cg_stream);
            for (Req *q : done) complete(q, q->failed ? CB_ERROR_HIP : CB_SUCCESS, q->iters, q->conv, q->rel);
            progressed = true;
        }
        // admission in arrival order; a solve waiting for the period's end lets SpMM requests pass,
        // a request waiting for memory holds everything behind it
        {
            std::unique_lock<std::mutex> lk(mu);
            for (auto it = pending.begin(); it != pending.end();) {
                Req *q = *it;
                lk.unlock();
                bool mem = false;
                const bool ok = admit_one(q, mem);
                lk.lock();
                if (ok) {
                    it = pending.erase(it);
                    progressed = true;
                } else if (mem) {
                    break;
                } else {
                    ++it;
                }
            }
            active_peak = std::max(active_peak, g64.active + g32.active + gmx.active);
        }
        // next period of the active solves
        if (!period_inflight && g64.active + g32.active + gmx.active > 0) {
            hipError_t e = enqueue_period();
            if (e != hipSuccess) {
                // fail every active solve
                std::vector<Req *> all;
                for (int i = 0; i < g64.top; ++i)
                    if (g64.req[i]) all.push_back(g64.req[i]), g64.req[i] = nullptr, g64.jobs[i].active = 0;
                for (int i = 0; i < g32.top; ++i)
                    if (g32.req[i]) all.push_back(g32.req[i]), g32.req[i] = nullptr, g32.jobs[i].active = 0;
                for (int i = 0; i < gmx.top; ++i)
                    if (gmx.req[i]) all.push_back(gmx.req[i]), gmx.req[i] = nullptr, gmx.jobs[i].active = 0;
                hipStreamSynchronize(cg_stream);
                g64.active = g32.active = gmx.active = g64.top = g32.top = gmx.top = 0;
                for (Req *q : all) complete(q, CB_ERROR_HIP, q->iters, 0, 0.0);
                dirty = true;
                hipGetLastError();
            } else {
                period_inflight = true;
            }
            progressed = true;
        }
        std::unique_lock<std::mutex> lk(mu);
        const bool busy = period_inflight || !spmm_inflight.empty();
        if (stop && pending.empty() && !busy && g64.active + g32.active + gmx.active == 0) break;
        if (!progressed) {
            if (busy || !pending.empty())
                cv_work.wait_for(lk, std::chrono::microseconds(20));
            else
                cv_work.wait_for(lk, std::chrono::milliseconds(50));
        }
    }
}

extern "C" {

cb_status_t cb_server_options_default(cb_server_options_t *opt) {
    if (!opt) return fail(CB_ERROR_INVALID_VALUE, "NULL options");
    *opt = cb_server_options_t{};
    opt->struct_size = sizeof(cb_server_options_t);
    opt->max_active = 64;
    opt->arena_bytes = (int64_t)1 << 30;
    opt->check_every = 8;
    opt->use_graph = 1;
    opt->spmm_streams = 2;
    return CB_SUCCESS;
}

cb_status_t cb_server_create(const cb_server_options_t *opt, cb_server_t *out) {
    if (!out) return fail(CB_ERROR_INVALID_VALUE, "NULL output");
    cb_server_options_t o;
    cb_server_options_default(&o);
    if (opt) {
        if (opt->struct_size != sizeof(cb_server_options_t))
            return fail(CB_ERROR_INVALID_VALUE, "cb_server_options_t.struct_size mismatch");
        o = *opt;
    }
    if (o.max_active < 1 || o.max_active > 4096 || o.arena_bytes < (int64_t)kAlign || o.check_every < 1 ||
        o.check_every > 1024 || (o.use_graph != 0 && o.use_graph != 1) || o.spmm_streams < 1 || o.spmm_streams > 16)
        return fail(CB_ERROR_INVALID_VALUE, "invalid server options");
    cb_server_s *S = new (std::nothrow) cb_server_s();
    if (!S) return fail(CB_ERROR_OUT_OF_MEMORY, "server");
    S->o = o;
    hipError_t e = hipGetDevice(&S->device);
    if (e == hipSuccess) e = hipMalloc(&S->arena_base, (size_t)o.arena_bytes);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        delete S;
        return fail(CB_ERROR_OUT_OF_MEMORY, "server arena");
    }
    if (e == hipSuccess) e = group_alloc(S->g64, o.max_active);
    if (e == hipSuccess) e = group_alloc(S->g32, o.max_active);
    if (e == hipSuccess) e = group_alloc(S->gmx, o.max_active);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->cg_stream, hipStreamNonBlocking);
    for (int i = 0; e == hipSuccess && i < o.spmm_streams; ++i) {
        hipStream_t s;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) S->spmm_streams.push_back(s);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->period_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        cb_server_destroy(S);
        return hipfail(e, "server creation");
    }
    S->arena.init((size_t)o.arena_bytes);
    S->mats.reserve(kMaxMatrices);
    S->worker = std::thread([S] { S->run(); });
    *out = S;
    return CB_SUCCESS;
}

cb_status_t cb_server_add_matrix(cb_server_t S, cb_matrix_t A, int32_t *id) {
    if (!S || !id) return fail(CB_ERROR_INVALID_VALUE, "NULL argument");
    Mat M{};
    M.A = A;
    cb_status_t st = cbh::matrix_view(A, M.v);
    if (st != CB_SUCCESS) return st;
    if (!M.v.natural) return fail(CB_ERROR_NOT_SUPPORTED, "the server runs natural-order structures (lb_mode contiguous or none)");
    if (M.v.device != S->device) return fail(CB_ERROR_NOT_SUPPORTED, "matrix on another device");
    M.esize = M.v.vector_f64 ? 8 : 4;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->mats.size() >= kMaxMatrices) return fail(CB_ERROR_NOT_SUPPORTED, "too many matrices");
    S->mats.push_back(M);
    *id = (int32_t)S->mats.size() - 1;
    return CB_SUCCESS;
}

cb_status_t cb_server_submit(cb_server_t S, const cb_request_t *req, int64_t *ticket) {
    if (!S || !req || !ticket) return fail(CB_ERROR_INVALID_VALUE, "NULL argument");
    if (req->struct_size != sizeof(cb_request_t)) return fail(CB_ERROR_INVALID_VALUE, "cb_request_t.struct_size mismatch");
    std::unique_lock<std::mutex> lk(S->mu);
    if (req->matrix < 0 || req->matrix >= (int32_t)S->mats.size()) return fail(CB_ERROR_INVALID_VALUE, "unknown matrix");
    const Mat &M = S->mats[req->matrix];
    if (req->kind != CB_REQ_SPMM && req->kind != CB_REQ_CG && req->kind != CB_REQ_CG_REFINE)
        return fail(CB_ERROR_INVALID_VALUE, "unknown request kind");
    const bool solve = req->kind != CB_REQ_SPMM;
    if (req->kind == CB_REQ_SPMM && req->k < 1) return fail(CB_ERROR_INVALID_VALUE, "k must be at least 1");
    if (solve && M.v.m != M.v.n) return fail(CB_ERROR_INVALID_VALUE, "CG needs a square matrix");
    if (solve && (req->rtol < 0.0 || req->max_iter < 0)) return fail(CB_ERROR_INVALID_VALUE, "invalid CG parameters");
    if (req->kind == CB_REQ_CG_REFINE) {
        if (M.v.vtype != CB_VALUE_F64) return fail(CB_ERROR_INVALID_VALUE, "a refined solve's matrix must store FP64 values");
        if (req->matrix_low < 0 || req->matrix_low >= (int32_t)S->mats.size())
            return fail(CB_ERROR_INVALID_VALUE, "unknown matrix_low");
        const Mat &L = S->mats[req->matrix_low];
        if ((L.v.vtype != CB_VALUE_F32 && L.v.vtype != CB_VALUE_BF16) || L.v.vector_f64)
            return fail(CB_ERROR_INVALID_VALUE, "matrix_low must store FP32 or BF16 values with float vectors");
        if (L.v.m != M.v.m || L.v.n != M.v.n) return fail(CB_ERROR_INVALID_VALUE, "matrix_low has another shape");
    }
    const bool need_in = M.v.n > 0, need_out = solve ? M.v.n > 0 : M.v.m > 0;
    if ((need_in && !req->in) || (need_out && !req->out)) return fail(CB_ERROR_INVALID_VALUE, "NULL vector");
    Req *q = new (std::nothrow) Req();
    if (!q) return fail(CB_ERROR_OUT_OF_MEMORY, "request");
    q->r = *req;
    q->pm = req->kind == CB_REQ_CG_REFINE ? req->matrix_low : req->matrix;
    q->anchor = -1.0;  // set from the first period's scalars
    q->rtol = req->rtol > 0.0 ? req->rtol : 1e-10;
    const int cap = req->max_iter > 0 ? req->max_iter : 500;
    q->max_iter = ((cap + S->o.check_every - 1) / S->o.check_every) * S->o.check_every;
    const size_t fp = footprint(q->r, M);
    ++S->submitted;
    if (fp > S->arena.size()) {
        ++S->rejected;
        delete q;
        return fail(CB_ERROR_OUT_OF_MEMORY, "request larger than the server's arena");
    }
    q->ticket = S->next_ticket++;
    q->t_submit = Clock::now();
    if (!S->started) {
        S->started = true;
        S->t_first = q->t_submit;
    }
    cb_response_t rs{};
    S->resp[q->ticket] = rs;
    S->pending.push_back(q);
    *ticket = q->ticket;
    lk.unlock();
    S->cv_work.notify_one();
    return CB_SUCCESS;
}

cb_status_t cb_server_poll(cb_server_t S, int64_t ticket, cb_response_t *resp) {
    if (!S || !resp) return fail(CB_ERROR_INVALID_VALUE, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->resp.find(ticket);
    if (it == S->resp.end()) return fail(CB_ERROR_INVALID_VALUE, "unknown ticket");
    *resp = it->second;
    return CB_SUCCESS;
}

cb_status_t cb_server_wait(cb_server_t S, int64_t ticket, cb_response_t *resp) {
    if (!S || !resp) return fail(CB_ERROR_INVALID_VALUE, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->resp.find(ticket);
    if (it == S->resp.end()) return fail(CB_ERROR_INVALID_VALUE, "unknown ticket");
    S->cv_done.wait(lk, [&] { return S->resp[ticket].done != 0; });
    *resp = S->resp[ticket];
    return CB_SUCCESS;
}

cb_status_t cb_server_stats(cb_server_t S, cb_server_stats_t *st) {
    if (!S || !st) return fail(CB_ERROR_INVALID_VALUE, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    cb_server_stats_t r{};
    r.submitted = S->submitted;
    r.rejected = S->rejected;
    r.completed = (int64_t)S->lat_us.size();
    r.spmm_done = S->spmm_done;
    r.cg_done = S->cg_done;
    if (!S->lat_us.empty()) {
        std::vector<double> v = S->lat_us;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const size_t i = (size_t)std::min<double>((double)v.size() - 1, std::ceil(p * (double)v.size()) - 1);
            return v[i];
        };
        r.p50_us = pct(0.50);
        r.p99_us = pct(0.99);
        double sum = 0.0;
        for (double x : v) sum += x;
        r.mean_us = sum / (double)v.size();
        r.elapsed_s = std::chrono::duration<double>(S->t_last - S->t_first).count();
        if (r.elapsed_s > 0.0) {
            r.requests_per_s = (double)r.completed / r.elapsed_s;
            r.solves_per_s = (double)r.cg_done / r.elapsed_s;
        }
    }
    r.arena_peak_bytes = (int64_t)S->arena.peak();
    r.active_peak = S->active_peak;
    r.graph_builds = S->graph_builds;
    r.steps = S->steps;
    *st = r;
    return CB_SUCCESS;
}

cb_status_t cb_server_destroy(cb_server_t S) {
    if (!S) return CB_SUCCESS;
    if (S->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv_work.notify_all();
        S->worker.join();
    }
    hipDeviceSynchronize();
    if (S->graph) hipGraphExecDestroy(S->graph);
    if (S->period_ev) hipEventDestroy(S->period_ev);
    for (hipStream_t s : S->spmm_streams) hipStreamDestroy(s);
    if (S->cg_stream) hipStreamDestroy(S->cg_stream);
    group_free(S->g64);
    group_free(S->g32);
    group_free(S->gmx);
    if (S->arena_base) hipFree(S->arena_base);
    delete S;
    return CB_SUCCESS;
}

}  // extern "C"
