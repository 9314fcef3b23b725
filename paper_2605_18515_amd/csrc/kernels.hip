// HIP kernels of libcbspmv for gfx950 (CDNA4, wave64).
//
// Work decomposition: one wavefront owns a contiguous range of tiles in kernel
// order (wave_ptr) and walks it tile by tile; four independent wavefronts
// share a 256-thread workgroup.  For every tile the wavefront
//   1. stages the 16 x values of the tile's columns in LDS (the tile's
//      column block, or the aggregated columns through restore_cols --
//      Section 3.5 preloads x in shared memory; with column aggregation the
//      16 original columns are gathered once per tile instead of per entry),
//   2. multiplies the tile's entries (Algorithm 3 for COO: one lane per
//      entry; CSR: four lanes per row with a DPP quad reduction, the wave64
//      form of the shuffle reduction of Section 3.5; Dense, Algorithm 4: four
//      lanes per row, four columns each, occupancy bits honoured),
//   3. adds the per-row sums into a 16-entry LDS accumulator for the panel.
// When the panel changes the accumulator is written to y: a plain store of
// alpha*sum + beta*y for panels owned by this wavefront, a global atomic add
// for panels shared with other wavefronts (pre-scaled by a pre-pass).
#include <hip/hip_runtime.h>

#include "cb_device.h"

namespace cbd {
namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlockThreads = kWave * kWavesPerBlock;

template <int VT>
struct Val;
template <>
struct Val<0> {
    using A = double;
    static constexpr int kSize = 8;
    __device__ static A load(const uint8_t *p, int i) { return reinterpret_cast<const double *>(p)[i]; }
};
template <>
struct Val<1> {
    using A = float;
    static constexpr int kSize = 4;
    __device__ static A load(const uint8_t *p, int i) { return reinterpret_cast<const float *>(p)[i]; }
};
template <>
struct Val<2> {
    using A = float;
    static constexpr int kSize = 2;
    __device__ static A load(const uint8_t *p, int i) {
        return __uint_as_float((uint32_t)reinterpret_cast<const uint16_t *>(p)[i] << 16);
    }
};

// Algorithm 3's padding between the one-byte indices and the values
__device__ __forceinline__ int pad_bytes(int index_bytes, int vsize) {
    const int r = index_bytes & (vsize - 1);
    return r ? vsize - r : 0;
}

// Workgroup b is dispatched to XCD b % 8.  Give each XCD a contiguous range of
// logical workgroups so neighbouring panels (which share x) meet in one L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b & 7, i = b >> 3, base = nb >> 3, extra = nb & 7;
    return x * base + (x < extra ? x : extra) + i;
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// sum over the four lanes of a quad (DPP quad_perm [1,0,3,2] then [2,3,0,1])
template <class A>
__device__ __forceinline__ A quad_sum(A v) {
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    return v;
}

template <class A>
__device__ __forceinline__ void lds_add(A *p, A v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

template <class A>
__device__ __forceinline__ void global_add(A *p, A v) {
    unsafeAtomicAdd(p, v);
}

template <int VT>
__global__ __launch_bounds__(kBlockThreads) void spmv_kernel(DevView d, typename Val<VT>::A alpha,
                                                              typename Val<VT>::A beta,
                                                              const typename Val<VT>::A *__restrict__ x,
                                                              typename Val<VT>::A *__restrict__ y) {
    using A = typename Val<VT>::A;
    constexpr int VS = Val<VT>::kSize;
    __shared__ A xs_all[kWavesPerBlock][16];
    __shared__ A acc_all[kWavesPerBlock][16];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int w = xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + wid;
    if (w >= d.nwaves) return;
    A *xs = xs_all[wid];
    A *acc = acc_all[wid];
    const int t0 = d.wave_ptr[w], t1 = d.wave_ptr[w + 1];
    if (lane < 16) acc[lane] = A(0);
    const int r4 = lane >> 2, q4 = lane & 3;

    auto flush = [&](int p) {
        if (lane < 16) {
            const int64_t row = 16 * (int64_t)p + lane;
            const A v = acc[lane];
            acc[lane] = A(0);
            if (row < d.m) {
                if (d.panel_shared[p]) {
                    global_add(&y[row], alpha * v);
                } else {
                    A r = alpha * v;
                    if (beta != A(0)) r += beta * y[row];
                    y[row] = r;
                }
            }
        }
    };

    int cur = -1;
    for (int t = t0; t < t1; ++t) {
        const int p = d.tile_row[t];
        const int c = d.tile_col[t];
        const int nz = d.tile_nnz[t];
        const int ty = d.tile_type[t];
        const uint8_t *base = d.payload + d.tile_vp[t];
        if (p != cur) {
            if (cur >= 0) flush(cur);
            cur = p;
        }
        if (lane < 16) {
            A xv = A(0);
            if (d.col_agg) {
                const int a = d.cols_offset[p] + 16 * c + lane;
                if (a < d.cols_offset[p + 1]) xv = x[d.restore_cols[a]];
            } else {
                const int64_t col = 16 * (int64_t)c + lane;
                if (col < d.n) xv = x[col];
            }
            xs[lane] = xv;
        }
        if (ty == 0) {
            const uint8_t *vals = base + nz + pad_bytes(nz, VS);
            for (int e = lane; e < nz; e += kWave) {
                const uint32_t code = base[e];
                lds_add(&acc[code & 15], Val<VT>::load(vals, e) * xs[code >> 4]);
            }
        } else if (ty == 1) {
            const uint8_t *codes = base + 16;
            const uint8_t *vals = codes + nz + pad_bytes(16 + nz, VS);
            const int s = base[r4];
            const int e_end = r4 < 15 ? (int)base[r4 + 1] : nz;
            A sum = A(0);
            for (int e = s + q4; e < e_end; e += 4) sum += Val<VT>::load(vals, e) * xs[codes[e] >> 4];
            sum = quad_sum(sum);
            if (q4 == 0) acc[r4] += sum;
        } else {
            const uint8_t *mask = base + 256 * VS;
            const uint32_t bits = (mask[2 * r4 + (q4 >> 1)] >> ((q4 & 1) * 4)) & 0xFu;
            A sum = A(0);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((bits >> j) & 1u) sum += Val<VT>::load(base, r4 * 16 + 4 * q4 + j) * xs[4 * q4 + j];
            sum = quad_sum(sum);
            if (q4 == 0) acc[r4] += sum;
        }
    }
    if (cur >= 0) flush(cur);
}

// k right-hand sides: KC columns of X per launch slice (blockIdx.y), 64 / KC
// entries in flight per wavefront pass, one lane per (entry, column).
template <int VT, int KC>
__global__ __launch_bounds__(kBlockThreads) void spmm_kernel(DevView d, typename Val<VT>::A alpha,
                                                              typename Val<VT>::A beta,
                                                              const typename Val<VT>::A *__restrict__ X, int64_t ldx,
                                                              typename Val<VT>::A *__restrict__ Y, int64_t ldy,
                                                              int k) {
    using A = typename Val<VT>::A;
    constexpr int VS = Val<VT>::kSize;
    constexpr int S = kWave / KC;
    __shared__ A xs_all[kWavesPerBlock][16 * KC];
    __shared__ A acc_all[kWavesPerBlock][16 * KC];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int w = xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + wid;
    if (w >= d.nwaves) return;
    const int j0 = blockIdx.y * KC;
    const int kc = min(KC, k - j0);
    A *xs = xs_all[wid];
    A *acc = acc_all[wid];
    const int t0 = d.wave_ptr[w], t1 = d.wave_ptr[w + 1];
    for (int i = lane; i < 16 * KC; i += kWave) acc[i] = A(0);
    const int slot = lane / KC, jj = lane % KC;

    auto flush = [&](int p) {
        const bool shared = d.panel_shared[p] != 0;
        for (int i = lane; i < 16 * KC; i += kWave) {
            const int r = i / KC, j = i % KC;
            const int64_t row = 16 * (int64_t)p + r;
            const A v = acc[i];
            acc[i] = A(0);
            if (row < d.m && j < kc) {
                A *yp = Y + row * ldy + j0 + j;
                if (shared) {
                    global_add(yp, alpha * v);
                } else {
                    A out = alpha * v;
                    if (beta != A(0)) out += beta * *yp;
                    *yp = out;
                }
            }
        }
    };

    int cur = -1;
    for (int t = t0; t < t1; ++t) {
        const int p = d.tile_row[t];
        const int c = d.tile_col[t];
        const int nz = d.tile_nnz[t];
        const int ty = d.tile_type[t];
        const uint8_t *base = d.payload + d.tile_vp[t];
        if (p != cur) {
            if (cur >= 0) flush(cur);
            cur = p;
        }
        for (int i = lane; i < 16 * KC; i += kWave) {
            const int lc = i / KC, j = i % KC;
            A xv = A(0);
            if (j < kc) {
                if (d.col_agg) {
                    const int a = d.cols_offset[p] + 16 * c + lc;
                    if (a < d.cols_offset[p + 1]) xv = X[(int64_t)d.restore_cols[a] * ldx + j0 + j];
                } else {
                    const int64_t col = 16 * (int64_t)c + lc;
                    if (col < d.n) xv = X[col * ldx + j0 + j];
                }
            }
            xs[i] = xv;
        }
        if (ty == 2) {
            const uint8_t *mask = base + 256 * VS;
            for (int e = slot; e < 256; e += S)
                if (((mask[e >> 3] >> (e & 7)) & 1u) && jj < kc)
                    lds_add(&acc[(e >> 4) * KC + jj], Val<VT>::load(base, e) * xs[(e & 15) * KC + jj]);
        } else {
            const int hdr = ty == 1 ? 16 : 0;
            const uint8_t *codes = base + hdr;
            const uint8_t *vals = codes + nz + pad_bytes(hdr + nz, VS);
            for (int e = slot; e < nz; e += S) {
                const uint32_t code = codes[e];
                if (jj < kc) lds_add(&acc[(code & 15) * KC + jj], Val<VT>::load(vals, e) * xs[(code >> 4) * KC + jj]);
            }
        }
    }
    if (cur >= 0) flush(cur);
}

// y <- beta * y (0 when beta == 0) on the rows of shared and empty panels
template <class A>
__global__ void prepass_kernel(const int32_t *__restrict__ list, int32_t np, int64_t m, A beta, A *__restrict__ y,
                               int k, int64_t ldy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = 16 * (int64_t)k;
    if (i >= (int64_t)np * per) return;
    const int64_t pi = i / per, rem = i - pi * per;
    const int64_t row = 16 * (int64_t)list[pi] + rem / k;
    const int j = (int)(rem % k);
    if (row >= m) return;
    A *yp = y + row * ldy + j;
    *yp = beta == A(0) ? A(0) : beta * *yp;
}

__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                   int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], e = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = e;
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

template <class A>
hipError_t prepass(const DevView &d, double beta, void *y, int k, int64_t ldy, hipStream_t s) {
    if (d.nprepass <= 0) return hipSuccess;
    const int64_t total = (int64_t)d.nprepass * 16 * k;
    const int64_t nb = (total + 255) / 256;
    hipLaunchKernelGGL(prepass_kernel<A>, dim3((unsigned)nb), dim3(256), 0, s, d.prepass_list, d.nprepass, d.m,
                       (A)beta, (A *)y, k, ldy);
    return hipGetLastError();
}

template <int VT>
hipError_t spmv_vt(const DevView &d, double alpha, const void *x, double beta, void *y, hipStream_t s) {
    using A = typename Val<VT>::A;
    hipError_t e = prepass<A>(d, beta, y, 1, 1, s);
    if (e != hipSuccess) return e;
    if (d.nwaves <= 0) return hipSuccess;
    const int nb = (d.nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL(spmv_kernel<VT>, dim3(nb), dim3(kBlockThreads), 0, s, d, (A)alpha, (A)beta, (const A *)x,
                       (A *)y);
    return hipGetLastError();
}

template <int VT, int KC>
hipError_t spmm_kc(const DevView &d, int k, double alpha, const void *X, int64_t ldx, double beta, void *Y,
                   int64_t ldy, hipStream_t s) {
    using A = typename Val<VT>::A;
    hipError_t e = prepass<A>(d, beta, Y, k, ldy, s);
    if (e != hipSuccess) return e;
    if (d.nwaves <= 0) return hipSuccess;
    const int nb = (d.nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
    const int ny = (k + KC - 1) / KC;
    hipLaunchKernelGGL((spmm_kernel<VT, KC>), dim3(nb, ny), dim3(kBlockThreads), 0, s, d, (A)alpha, (A)beta,
                       (const A *)X, ldx, (A *)Y, ldy, k);
    return hipGetLastError();
}

template <int VT>
hipError_t spmm_vt(const DevView &d, int k, double alpha, const void *X, int64_t ldx, double beta, void *Y,
                   int64_t ldy, hipStream_t s) {
    if (k <= 1) return spmm_kc<VT, 1>(d, k, alpha, X, ldx, beta, Y, ldy, s);
    if (k <= 2) return spmm_kc<VT, 2>(d, k, alpha, X, ldx, beta, Y, ldy, s);
    if (k <= 4) return spmm_kc<VT, 4>(d, k, alpha, X, ldx, beta, Y, ldy, s);
    if (k <= 8) return spmm_kc<VT, 8>(d, k, alpha, X, ldx, beta, Y, ldy, s);
    if (k <= 16) return spmm_kc<VT, 16>(d, k, alpha, X, ldx, beta, Y, ldy, s);
    return spmm_kc<VT, 32>(d, k, alpha, X, ldx, beta, Y, ldy, s);
}

}  // namespace

hipError_t launch_spmv(const DevView &d, int vtype, double alpha, const void *x, double beta, void *y,
                       hipStream_t stream) {
    switch (vtype) {
        case 0: return spmv_vt<0>(d, alpha, x, beta, y, stream);
        case 1: return spmv_vt<1>(d, alpha, x, beta, y, stream);
        case 2: return spmv_vt<2>(d, alpha, x, beta, y, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spmm(const DevView &d, int vtype, int k, double alpha, const void *X, int64_t ldx, double beta,
                       void *Y, int64_t ldy, hipStream_t stream) {
    switch (vtype) {
        case 0: return spmm_vt<0>(d, k, alpha, X, ldx, beta, Y, ldy, stream);
        case 1: return spmm_vt<1>(d, k, alpha, X, ldx, beta, Y, ldy, stream);
        case 2: return spmm_vt<2>(d, k, alpha, X, ldx, beta, Y, ldy, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t stream) {
    const int64_t n16 = bytes / 16;
    int64_t nb = (n16 + 255) / 256;
    if (nb > 8192) nb = 8192;
    if (nb < 1) return hipSuccess;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)nb), dim3(256), 0, stream, (const uint4 *)src, (uint4 *)dst, n16);
    return hipGetLastError();
}

}  // namespace cbd
