// HIP kernels of libcbspmv for gfx950 (CDNA4, wave64).
//
// Work decomposition: one wavefront owns a contiguous range of tiles in kernel
// order (wave_ptr); four independent wavefronts share a 256-thread workgroup,
// and workgroups are remapped so that each XCD takes a contiguous eighth of the
// ranges (neighbouring panels share x in one L2).
//   spmv_stream_kernel  natural order (contiguous or no load balance): streams
//                       the range's payload and the converter's batch records
//                       through a four-stage pipeline, multiplying the COO and
//                       CSR entries of a batch as one stream (below).
//   spmv_kernel         Algorithm 2 order: one tile at a time -- the tile's 16
//                       x values staged in LDS (Section 3.5; through
//                       restore_cols under column aggregation, once per tile
//                       instead of per entry), COO one lane per entry
//                       (Algorithm 3), CSR and Dense four lanes per row with a
//                       DPP quad reduction (Algorithm 4's shuffle reduction).
//   spmm_kernel         k right-hand sides, KC columns per launch slice, Dense
//                       tiles on the matrix cores.
// Row sums accumulate per panel in LDS and are written to y once per panel: a
// plain store of alpha*sum + beta*y for panels owned by the wavefront, a global
// atomic add for panels shared with other wavefronts (pre-scaled by a pre-pass).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "cb_device.h"
#include "cb_stream.h"

namespace cbd {
namespace {

// Tuning parameters (fixed at build time; the defaults are the measured best on MI355X)
#ifndef CB_TUNE_WAVES_PER_BLOCK
#define CB_TUNE_WAVES_PER_BLOCK 1
#endif
#ifndef CB_TUNE_PASS_PAIRS
#define CB_TUNE_PASS_PAIRS 1  // flat entry passes two at a time (FP32/BF16 values)
#endif
#ifndef CB_TUNE_SPMM_MFMA
#define CB_TUNE_SPMM_MFMA 1  // natural-order SpMM on the matrix cores (0: the tile-at-a-time kernel)
#endif
#ifndef CB_TUNE_SPMM_STAGES
#define CB_TUNE_SPMM_STAGES 2  // tiles whose loads are in flight in the matrix-core SpMM (FP64: one fewer, at least 2)
#endif
#ifndef CB_TUNE_SPMM_KC_MAX
#define CB_TUNE_SPMM_KC_MAX 32  // widest column slice of the matrix-core SpMM (16 or 32)
#endif
#ifndef CB_TUNE_NT_LOADS
#define CB_TUNE_NT_LOADS 0  // payload chunk loads with the nontemporal hint
#endif
#ifndef CB_TUNE_QCPOL
#define CB_TUNE_QCPOL 0  // cache-policy bits of the quad kernel's payload and record loads (2: nontemporal)
#endif

// a load of streamed (read-once) data, with the nontemporal hint when NT
template <bool NT, class T>
__device__ __forceinline__ T ld_stream(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

constexpr int kWave = 64;
constexpr int kWavesPerBlock = CB_TUNE_WAVES_PER_BLOCK;
constexpr int kBlockThreads = kWave * kWavesPerBlock;

template <int VT>
struct Val;
// load(p, i): value i of a packed value array; load4(p, i, v): values i .. i+3 (i a multiple of 4,
// the array aligned to its value size) with the widest loads the alignment allows
template <>
struct Val<0> {
    using A = double;
    static constexpr int kSize = 8;
    __device__ static A load(const uint8_t *p, int i) { return reinterpret_cast<const double *>(p)[i]; }
    __device__ static void load4(const uint8_t *p, int i, A *v) {
        using d2 = double __attribute__((ext_vector_type(2), aligned(8)));
        const d2 a = *reinterpret_cast<const d2 *>(p + 8 * i), b = *reinterpret_cast<const d2 *>(p + 8 * i + 16);
        v[0] = a.x;
        v[1] = a.y;
        v[2] = b.x;
        v[3] = b.y;
    }
};
template <>
struct Val<1> {
    using A = float;
    static constexpr int kSize = 4;
    __device__ static A load(const uint8_t *p, int i) { return reinterpret_cast<const float *>(p)[i]; }
    __device__ static void load4(const uint8_t *p, int i, A *v) {
        using f4 = float __attribute__((ext_vector_type(4), aligned(4)));
        const f4 a = *reinterpret_cast<const f4 *>(p + 4 * i);
        v[0] = a.x;
        v[1] = a.y;
        v[2] = a.z;
        v[3] = a.w;
    }
};
template <>
struct Val<2> {
    using A = float;
    static constexpr int kSize = 2;
    __device__ static A load(const uint8_t *p, int i) {
        return __uint_as_float((uint32_t)reinterpret_cast<const uint16_t *>(p)[i] << 16);
    }
    __device__ static void load4(const uint8_t *p, int i, A *v) {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = load(p, i + j);
    }
};
// FP32 / BF16 values with double vectors: the stored value widened exactly, FP64 arithmetic
template <>
struct Val<3> {
    using A = double;
    static constexpr int kSize = 4;
    __device__ static A load(const uint8_t *p, int i) { return (double)Val<1>::load(p, i); }
    __device__ static void load4(const uint8_t *p, int i, A *v) {
        float f[4];
        Val<1>::load4(p, i, f);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (double)f[j];
    }
};
template <>
struct Val<4> {
    using A = double;
    static constexpr int kSize = 2;
    __device__ static A load(const uint8_t *p, int i) { return (double)Val<2>::load(p, i); }
    __device__ static void load4(const uint8_t *p, int i, A *v) {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = load(p, i + j);
    }
};

// Algorithm 3's padding between the one-byte indices and the values
__device__ __forceinline__ int pad_bytes(int index_bytes, int vsize) {
    const int r = index_bytes & (vsize - 1);
    return r ? vsize - r : 0;
}

// Byte of a device array at a wave-uniform index, read through the scalar cache as the
// aligned dword that holds it (sub-arrays start on 256-byte boundaries, so the dword lies
// inside the allocation).
__device__ __forceinline__ int uniform_byte(const uint8_t *p, int64_t i) {
    const uint32_t w = reinterpret_cast<const uint32_t *>(p)[i >> 2];
    return (int)((w >> (8 * (i & 3))) & 0xFFu);
}

// Workgroup b is dispatched to XCD b % 8.  chunk c >= 1: XCD x takes runs of c consecutive work
// ranges, the eight XCDs side by side (x c .. x c + c - 1 of every 8 c ranges; the last partial
// group of 8 c in dispatch order); c = 0: each XCD a contiguous eighth of the ranges.
__device__ __forceinline__ int xcd_block(int b, int nb, int c) {
    const int x = b & 7, i = b >> 3;
    if (c <= 0) {
        const int base = nb >> 3, extra = nb & 7;
        return x * base + (x < extra ? x : extra) + i;
    }
    const int64_t g0 = (int64_t)(i / c) * (8 * (int64_t)c);
    if (g0 + 8 * (int64_t)c > nb) return b;
    return (int)g0 + x * c + i % c;
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

// DPP move with `old` returned where the source lane lies outside the 16-lane row
template <int CTRL>
__device__ __forceinline__ int dpp_or(int v, int old) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_or(float v, float old) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_or(double v, double old) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <class A>
__device__ __forceinline__ void lds_add(A *p, A v);

// Adds each lane's product into *dst, where lanes with equal keys share dst and
// equal keys occupy consecutive lanes (entries in (tile, row) order).  A
// segmented inclusive scan inside every 16-lane DPP row (row_shr 1, 2, 4, 8)
// leaves each run's sum in its last lane; only those lanes add, so an
// accumulator meets at most one add per run.  Lanes without an entry carry a
// key no other lane has.
template <class A>
__device__ __forceinline__ void segmented_row_add(A val, int key, bool valid, A *dst) {
    int kp;
    A vp;
    kp = dpp_or<0x111>(key, -1);
    vp = dpp_or<0x111>(val, A(0));
    if (kp == key) val += vp;
    kp = dpp_or<0x112>(key, -1);
    vp = dpp_or<0x112>(val, A(0));
    if (kp == key) val += vp;
    kp = dpp_or<0x114>(key, -1);
    vp = dpp_or<0x114>(val, A(0));
    if (kp == key) val += vp;
    kp = dpp_or<0x118>(key, -1);
    vp = dpp_or<0x118>(val, A(0));
    if (kp == key) val += vp;
    const int kn = dpp_or<0x101>(key, -2);  // row_shl:1, the next lane's key
    if (valid && kn != key) lds_add(dst, val);
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
    const int w = xcd_block(blockIdx.x, gridDim.x, d.xcd_chunk) * kWavesPerBlock + wid;
    if (w >= d.nwaves) return;
    A *xs = xs_all[wid];
    A *acc = acc_all[wid];
    const int t0 = d.wave_ptr[w], t1 = d.wave_ptr[w + 1];
    // tile size S = 16 or 8: rows of a panel, columns of a tile; CSR and Dense tiles take four lanes
    // per row (lanes of rows past S idle), S / 4 values per lane of a Dense row
    const int LT = d.tile_lt, S = 1 << LT, vpl = S >> 2;
    if (lane < 16) acc[lane] = A(0);
    const int r4 = lane >> 2, q4 = lane & 3;

    auto flush = [&](int p) {
        if (lane < S) {
            const int64_t row = ((int64_t)p << LT) + lane;
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
        if (lane < S) {
            A xv = A(0);
            if (d.col_agg) {
                const int a = d.cols_offset[p] + (c << LT) + lane;
                if (a < d.cols_offset[p + 1]) xv = x[d.restore_cols[a]];
            } else {
                const int64_t col = ((int64_t)c << LT) + lane;
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
            const uint8_t *codes = base + S;
            const uint8_t *vals = codes + nz + pad_bytes(S + nz, VS);
            A sum = A(0);
            if (r4 < S) {
                const int s = base[r4];
                const int e_end = r4 < S - 1 ? (int)base[r4 + 1] : nz;
                for (int e = s + q4; e < e_end; e += 4) sum += Val<VT>::load(vals, e) * xs[codes[e] >> 4];
            }
            sum = quad_sum(sum);
            if (q4 == 0 && r4 < S) acc[r4] += sum;
        } else {
            // Dense: lane (r4, q4) takes elements e0 .. e0 + S/4 - 1 of row r4, e0 = r4 S + q4 S / 4
            const uint8_t *mask = base + (S * S) * VS;
            const int e0 = (r4 << LT) + q4 * vpl;
            const uint32_t bits = r4 < S ? (mask[e0 >> 3] >> (e0 & 7)) & ((1u << vpl) - 1u) : 0u;
            A sum = A(0);
            for (int j = 0; j < vpl; ++j)
                if ((bits >> j) & 1u) sum += Val<VT>::load(base, e0 + j) * xs[q4 * vpl + j];
            sum = quad_sum(sum);
            if (q4 == 0 && r4 < S) acc[r4] += sum;
        }
    }
    if (cur >= 0) flush(cur);
}

// ---- streaming SpMV over natural-order structures --------------------------
//
// When the kernel order equals the packing order (contiguous or no load
// balance), a wavefront's tiles occupy one contiguous byte range of the
// payload.  The converter cuts the range into batches (at most 16 tiles whose
// payload touches at most four 1 KB chunks and whose panels lie within four
// consecutive ones) and writes each batch as a header and one record per tile
// (format in cb_stream.h): the offsets the multiply needs, precomputed once.
// The loads of a batch are spread over the three steps before the one that
// multiplies it, so every step waits once, at its top, for loads issued one
// step earlier:
//   step b-3  issues batch b's header and records (one 16-byte load per lane),
//   step b-2  stores them in LDS and issues the loads of the batch's x column
//             indices (under column aggregation the tiles' original columns,
//             tile_cols, 64 contiguous bytes per tile; else the column blocks),
//   step b-1  issues batch b's payload chunks and its x values,
//   step b    moves both into LDS and multiplies the batch.
// The multiply treats the COO and CSR tiles of a batch as one stream of
// entries -- both formats store a one-byte (row, column) code per entry,
// Algorithm 3 -- so lane i of pass p takes entry 64p+i whatever tile it is
// in, finds its tile from the tiles' end positions, and adds value * x into
// the LDS accumulator of its panel row.  Dense tiles (Algorithm 4) are
// multiplied one at a time, four lanes per row.  A panel is written to y at
// the top of the step after its last tile was multiplied (alpha*sum + beta*y,
// y read one step ahead; a global atomic add for panels shared with another
// wavefront, pre-scaled by a pre-pass).

using u32x4 = unsigned int __attribute__((ext_vector_type(4)));
using i32x4 = int __attribute__((ext_vector_type(4)));
using i32x2 = int __attribute__((ext_vector_type(2)));

constexpr int kChunk = cbs::kChunk;
constexpr int kRC = cbs::kRingChunks;
constexpr int kPRing = kRC * kChunk;  // payload ring per wavefront
constexpr int kPMask = kPRing - 1;
constexpr int kBatchTiles = cbs::kBatchTiles;
constexpr int kMaxPanels = cbs::kBatchPanels;
static_assert(kChunk == kWave * 16 && (kPRing & kPMask) == 0, "one chunk per wavefront-wide 16-byte load");
static_assert(kBatchTiles + 1 <= kWave && kBatchTiles % 4 == 0, "a batch's records fit one load; x gathers take four tiles each");
static_assert(kMaxPanels * 16 <= kWave && kMaxPanels <= 4, "accumulators cleared by one store per lane, flushed by one group");
constexpr int kWaitVm0 = 0x0F70;  // s_waitcnt vmcnt(0), expcnt and lgkmcnt left at their maxima

// RR, the row sums: 0 = one LDS atomic add per entry, 1 = DPP segmented scan then one add per run,
// 2 = one FP64 LDS atomic add per entry (FP32/BF16 values: the products widened, the row sums kept
// in FP64 until they are written), 3 and 4 = 0 and 2 with two copies of the accumulators, odd lanes
// adding into the second (entries of a row sit in neighbouring lanes, so long rows collide half as
// often on one LDS address; the copies are added when the panel is written)
// One work range w of the structure d (the body of the streaming kernel, shared by the one-matrix
// and the batched launch).  LT: log2 of the tile size S (4: 16 x 16 tiles, 3: 8 x 8).
template <int VT, int AGG, int RR, int LT>
__device__ __forceinline__ void stream_range(const DevView &d, int w, typename Val<VT>::A alpha,
                                             typename Val<VT>::A beta, const typename Val<VT>::A *__restrict__ x,
                                             typename Val<VT>::A *__restrict__ y) {
    using A = typename Val<VT>::A;
    constexpr int S = 1 << LT;  // rows of a panel, columns of a tile
    constexpr int TPG = kWave / S;  // tiles per x gather
    static_assert(LT == 3 || LT == 4, "16 x 16 or 8 x 8 tiles");
    static_assert(AGG >= 0 && AGG <= 2, "per-batch column bases are a quad-batch form");
    using AC = typename std::conditional<RR == 2 || RR == 4, double, A>::type;  // accumulator type
    constexpr bool DPPRED = RR == 1;
    constexpr int NACC = RR >= 3 ? 2 : 1;  // accumulator copies
    constexpr int VS = Val<VT>::kSize;
    __shared__ __align__(16) uint8_t pring_all[kWavesPerBlock][kPRing];
    __shared__ __align__(16) A xarea_all[kWavesPerBlock][kBatchTiles * S];
    __shared__ __align__(16) AC acc_all[kWavesPerBlock][kMaxPanels * 16 * NACC];
    const int lane = threadIdx.x & (kWave - 1);
    // with one wavefront per workgroup its LDS arrays sit at fixed addresses
    const int wid = kWavesPerBlock == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (w >= d.nwaves) return;
    const int o_begin = d.batch_ptr[w], o_end = d.batch_ptr[w + 1];
    if (o_begin >= o_end) return;
    uint8_t *pring = pring_all[wid];
    A *xarea = xarea_all[wid];
    AC *acc = acc_all[wid];
    const int t0 = d.wave_ptr[w], t1 = d.wave_ptr[w + 1];
    const u32x4 *pstream = reinterpret_cast<const u32x4 *>(d.payload + d.tile_vp[t0]) + lane;
    const i32x4 *rstream = reinterpret_cast<const i32x4 *>(d.batch_stream);
    // only the first and the last panel of a natural-order range can be shared with another range
    const int p_first = d.tile_row[t0], p_last = d.tile_row[t1 - 1];
    const bool sh_first = d.panel_shared[p_first] != 0, sh_last = d.panel_shared[p_last] != 0;
    const int gj = lane >> LT, glc = lane & (S - 1);

    // header and records of the batch at record o: lane i < 16 record i (lanes 16 .. 62 record 15
    // again), lane 63 the header.  Three batches' records stay in registers, one tile per lane:
    // {record word, last flat entry (COO/CSR) or region start (Dense)}, never both set
    i32x4 Q;
    auto qload = [&](int o) {
        Q = ld_stream<CB_TUNE_NT_LOADS != 0>(&rstream[o + (lane == kWave - 1 ? 0 : 1 + min(lane, kBatchTiles - 1))]);
    };
    auto recv = [&]() { return i32x2{Q.x, Q.y | Q.z}; };

    // payload chunks of a batch not loaded yet (chi: chunks whose loads were issued); re is the
    // batch's end, and it starts where the previous batch ended
    u32x4 P[kRC];
    int chi = 0, pfirst = 0, pcnt = 0;
    auto issue_payload = [&](int re) {
        const int lastc = (re - 1) >> 10;
        pfirst = chi;
        pcnt = lastc - chi + 1;
#pragma unroll
        for (int i = 0; i < kRC; ++i) {
            if (i < pcnt) {
                const u32x4 *src = pstream + (size_t)(chi + i) * kWave;
                P[i] = CB_TUNE_NT_LOADS ? __builtin_nontemporal_load(src) : *src;
            }
        }
        chi = max(chi, lastc + 1);
    };
    auto put_payload = [&]() {
        u32x4 *ring4 = reinterpret_cast<u32x4 *>(pring);
#pragma unroll
        for (int i = 0; i < kRC; ++i)
            if (i < pcnt) ring4[((pfirst + i) & (kRC - 1)) * kWave + lane] = P[i];
    };
    // x of a batch whose first tile is tb (nt tiles): in gather g, lane (gj, glc) takes column glc of
    // tile tb + TPG g + gj (clamped to the range), so x lands at x area entry S * (tile in batch) +
    // glc.  The column indices are loaded one step before the x values: under aggregation the tiles'
    // original columns (tile_cols, 256 contiguous bytes per gather), else the tiles' column blocks.
    // Columns past a tile's last one read a valid column of the matrix and are never multiplied.
    // Compressed columns (AGG 2): the lane's 2-byte offset and its tile's base, both vector loads (a
    // scalar load would make every later LDS read wait for it: the two share one counter).
    constexpr int NG = (kBatchTiles + TPG - 1) / TPG;
    int RG[NG];
    int RB[NG];
    auto issue_cols = [&](int tb, int nt) {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (TPG * g < nt) {
                const int t = min(tb + TPG * g + gj, t1 - 1);
                if constexpr (AGG == 2) {
                    RG[g] = (int)ld_stream<CB_TUNE_NT_LOADS != 0>(&d.tile_c16[S * (size_t)t + glc]);
                    RB[g] = ld_stream<CB_TUNE_NT_LOADS != 0>(&d.tile_cbase[t]);
                } else {
                    RG[g] = AGG ? ld_stream<CB_TUNE_NT_LOADS != 0>(&d.tile_cols[S * (size_t)t + (glc & 3) * (S / 4) + (glc >> 2)])
                                : d.tile_col[t];
                }
            }
        }
    };
    A XG[NG];
    auto issue_x = [&](int nt) {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (TPG * g < nt) {
                int col = RG[g];
                if constexpr (AGG == 2) {
                    col += RB[g];
                } else if constexpr (!AGG) {
                    const int64_t c = S * (int64_t)RG[g] + glc;
                    col = c < d.n ? (int)c : 0;
                }
                XG[g] = x[col];
            }
        }
    };
    auto put_x = [&](int nt) {
#pragma unroll
        for (int g = 0; g < NG; ++g)
            if (TPG * g < nt) xarea[64 * g + lane] = XG[g];
    };

    // panels finished by a batch: lane (k, r) holds row r of panel pb + k (rows r < S)
    const int fk = lane >> 4, fr = lane & 15;
    A YP = A(0);
    int done_pb = 0, done_mask = 0;
    auto is_shared = [&](int p) { return (p == p_first && sh_first) || (p == p_last && sh_last); };
    auto issue_y = [&]() {
        if (beta == A(0)) return;
        const int64_t row = S * (int64_t)(done_pb + fk) + fr;
        if (((done_mask >> fk) & 1) && fr < S && row < d.m && !is_shared(done_pb + fk)) YP = y[row];
    };
    auto flush = [&]() {
        if ((done_mask >> fk) & 1) {
            const int p = done_pb + fk;
            AC *a = &acc[(p & (kMaxPanels - 1)) * 16 * NACC + fr];
            AC sv = *a;
            *a = AC(0);
            if constexpr (NACC == 2) {
                sv += a[16];
                a[16] = AC(0);
            }
            const A v = (A)sv;
            const int64_t row = S * (int64_t)p + fr;
            if (fr < S && row < d.m) {
                if (is_shared(p)) {
                    global_add(&y[row], alpha * v);
                } else {
                    A r = alpha * v;
                    if (beta != A(0)) r += beta * YP;
                    y[row] = r;
                }
            }
        }
        done_mask = 0;
    };

    // multiply one batch: its records in rl (lane i holds tile i's), header fields hz = nt | nflat << 8 |
    // ndense << 16 | done << 24 and etot (flat entries); positions in the packed record words are taken
    // modulo the ring size
    auto multiply = [&](const i32x2 rl, int hz, int etot) {
        const int nflat = (hz >> 8) & 0xFF, ndense = (hz >> 16) & 0xFF;
        // COO and CSR entries as one stream; lane i holds flat tile i's last entry (endv) and record
        // word (pkv); lanes from nflat on hold the last flat tile's word, which the lanes past the
        // batch's last entry select (their tile position then stays inside the x area)
        const int endv = rl.y;
        const uint32_t pkv =
            lane < nflat ? (uint32_t)rl.x : (uint32_t)__builtin_amdgcn_readlane(rl.x, nflat > 0 ? nflat - 1 : 0);
        // pass (64 entries) holding each flat tile's last entry
        const int passv = lane < nflat ? endv / kWave : -1;
        // tile of entry E in the pass starting at entry e0 (a multiple of 64), and its record word;
        // j: the tile holding entry e0, advanced to the tile holding entry e0 + 64.  The tiles that
        // end inside the pass are j, j + 1, ...: their number comes from one ballot, and only they
        // are walked (selects, not branches, keep the walk uniform)
        auto tile_of = [&](int e0, int E, int &j, uint32_t &pk) {
            int ti = j;
            pk = __builtin_amdgcn_readlane(pkv, min(j, kBatchTiles - 1));
            const int c = __builtin_popcountll(__builtin_amdgcn_ballot_w64(passv == e0 / kWave));
            for (int k = 0; k < c; ++k) {
                const int i = j + k;
                const int ei = __builtin_amdgcn_readlane(endv, i);
                // i + 1 <= 16: lanes from kBatchTiles on hold the last record again
                const uint32_t pn = __builtin_amdgcn_readlane(pkv, i + 1);
                const bool past = E > ei;
                ti += past ? 1 : 0;
                pk = past ? pn : pk;
            }
            j += c;
            return ti;
        };
        // one entry: code, value and x through the tile's packed record word
        auto entry = [&](uint32_t pk, int E, uint32_t &code) {
            code = pring[(pk + E) & kPMask];
            return Val<VT>::load(pring + (((pk >> cbs::kRingBits) + VS * E) & kPMask), 0) *
                   xarea[((pk >> 27) << LT) + (code >> 4)];
        };
        auto accumulate = [&](A prod, int ti, uint32_t code, uint32_t pk, bool valid) {
            const int slot = (pk >> 24) & (kMaxPanels - 1);
            AC *dst = &acc[slot * 16 * NACC + (NACC == 2 ? (lane & 1) << 4 : 0) + (code & 15)];
            if constexpr (DPPRED) {
                segmented_row_add(valid ? prod : A(0), valid ? (ti << 4) | (int)(code & 15) : 0x10000 + lane, valid,
                                  dst);
            } else if (valid) {
                lds_add(dst, (AC)prod);
            }
        };
        int j = 0;
        int e0 = 0;
        // two passes at a time, their LDS reads interleaved (each pass is a chain of two dependent
        // reads: code, then x); the first pass of a pair is full.  Measured faster with the DPP
        // reduction of FP32/BF16 sums and not with FP64 LDS atomics.
        for (; CB_TUNE_PASS_PAIRS && DPPRED && e0 + kWave < etot; e0 += 2 * kWave) {
            const int Ea = e0 + lane, Eb = Ea + kWave;
            uint32_t pa, pb;
            const int ta = tile_of(e0, Ea, j, pa);
            const int tb = tile_of(e0 + kWave, Eb, j, pb);
            uint32_t ca, cb;
            const A prod_a = entry(pa, Ea, ca), prod_b = entry(pb, Eb, cb);
            accumulate(prod_a, ta, ca, pa, true);
            accumulate(prod_b, tb, cb, pb, Eb < etot);
        }
        // full passes, then the partial one: only the last pass needs the lane mask
        const int efull = etot & ~(kWave - 1);
        for (; e0 < efull; e0 += kWave) {
            const int E = e0 + lane;
            uint32_t pk;
            const int ti = tile_of(e0, E, j, pk);
            uint32_t code;
            const A prod = entry(pk, E, code);
            accumulate(prod, ti, code, pk, true);
        }
        if (e0 < etot) {
            const int E = e0 + lane;
            uint32_t pk;
            const int ti = tile_of(e0, E, j, pk);
            uint32_t code;
            const A prod = entry(pk, E, code);
            accumulate(prod, ti, code, pk, E < etot);
        }
        // dense tiles, four lanes per row: lane (r4, q4) takes elements ed .. ed + S/4 - 1 of row r4,
        // ed = r4 S + q4 S / 4, under its bits of the occupancy bitmap (rows past S idle)
        constexpr int VPL = S / 4;
        const int r4 = lane >> 2, q4 = lane & 3;
        const int ed = (r4 << LT) + q4 * VPL;
        for (int k = 0; k < ndense; ++k) {
            const uint32_t pk = (uint32_t)__builtin_amdgcn_readlane(rl.x, nflat + k);
            const int rel = __builtin_amdgcn_readlane(rl.y, nflat + k);
            const uint32_t bits =
                r4 < S ? (pring[(rel + S * S * VS + (ed >> 3)) & kPMask] >> (ed & 7)) & ((1u << VPL) - 1u) : 0u;
            const int vo = rel + ed * VS;
            const A *xs = xarea + ((pk >> 27) << LT) + VPL * q4;
            A sum = A(0);
#pragma unroll
            for (int jj = 0; jj < VPL; ++jj)
                if ((bits >> jj) & 1u) sum += Val<VT>::load(pring + ((vo + jj * VS) & kPMask), 0) * xs[jj];
            sum = quad_sum(sum);
            if (q4 == 0 && r4 < S) lds_add(&acc[((pk >> 24) & (kMaxPanels - 1)) * 16 * NACC + r4], (AC)sum);
        }
    };

    if (lane < kMaxPanels * 16) acc[lane] = AC(0);
    if constexpr (NACC == 2) acc[lane + 64] = AC(0);
    // Prologue: batch 0's records, x columns, x values and payload; batch 1's records and x
    // columns; batch 2's records.  At the top of step b the registers hold P and XG of batch b,
    // RG of batch b+1 and Q of batch b+2, and R0, R1 the records of batches b and b+1.
    // header fields of a batch: hz (nt | nflat << 8 | ndense << 16 | done << 24), etot, first panel
    struct Hdr {
        int re, hz, etot, pb;
    };
    auto header = [&]() {
        return Hdr{__builtin_amdgcn_readlane(Q.x, kWave - 1), __builtin_amdgcn_readlane(Q.z, kWave - 1),
                   __builtin_amdgcn_readlane(Q.w, kWave - 1), __builtin_amdgcn_readlane(Q.y, kWave - 1)};
    };
    int ob = o_begin;
    qload(ob);
    Hdr h0 = header(), h1{}, h2{};
    int ntb = h0.hz & 0xFF;
    i32x2 R0 = recv(), R1{}, R2{};
    issue_cols(t0, ntb);
    issue_payload(h0.re);
    int o1 = ob + 1 + ntb, nt1 = 0;
    const int tb1 = t0 + ntb;
    if (o1 < o_end) qload(o1);
    issue_x(ntb);  // waits for batch 0's x columns
    int o2 = o1, tb2 = tb1;
    if (o1 < o_end) {
        h1 = header();
        nt1 = h1.hz & 0xFF;
        R1 = recv();
        issue_cols(tb1, nt1);
        o2 = o1 + 1 + nt1;
        tb2 = tb1 + nt1;
        if (o2 < o_end) qload(o2);
    }
    while (ob < o_end) {
        // the one wait of a step: every load issued by the previous step has landed (loads are
        // issued conditionally, so the compiler's own counting would wait inside step 2)
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        // 1. payload and x of batch b into LDS, the panels batch b-1 finished to y, batch b+2's records
        put_payload();
        put_x(ntb);
        flush();
        const bool have1 = o1 < o_end, have2 = o2 < o_end;
        int nt2 = 0, o3 = o2;
        if (have2) {
            h2 = header();
            nt2 = h2.hz & 0xFF;
            R2 = recv();
        }
        __builtin_amdgcn_wave_barrier();
        // 2. loads: payload and x of batch b+1, x columns of batch b+2, records of batch b+3, and
        //    y of the panels batch b finishes
        if (have1) {
            issue_payload(h1.re);
            issue_x(nt1);
        }
        if (have2) {
            issue_cols(tb2, nt2);
            o3 = o2 + 1 + nt2;
            if (o3 < o_end) qload(o3);
        }
        done_pb = h0.pb;
        done_mask = (int)((uint32_t)h0.hz >> 24);
        issue_y();
        // 3. batch b
        multiply(R0, h0.hz, h0.etot);
        __builtin_amdgcn_wave_barrier();
        ob = o1;
        ntb = nt1;
        h0 = h1;
        o1 = o2;
        nt1 = nt2;
        h1 = h2;
        o2 = o3;
        tb2 += nt2;
        R0 = R1;
        R1 = R2;
    }
    flush();
}

template <int VT, int AGG, int RR, int LT>
__global__ __launch_bounds__(kBlockThreads) void spmv_stream_kernel(DevView d, typename Val<VT>::A alpha,
                                                                     typename Val<VT>::A beta,
                                                                     const typename Val<VT>::A *__restrict__ x,
                                                                     typename Val<VT>::A *__restrict__ y) {
    const int wid = kWavesPerBlock == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    stream_range<VT, AGG, RR, LT>(d, xcd_block(blockIdx.x, gridDim.x, d.xcd_chunk) * kWavesPerBlock + wid, alpha, beta,
                                  x, y);
}

// Products of several matrices in one launch (the serving loop's batches): workgroup b, after the
// XCD remap, runs work range b - jobs[j].wave_base of job j = wave_job[b]; every job of a launch has
// the same value type, aggregation, row-sum mode and tile size.
template <int VT, int AGG, int RR, int LT>
__global__ __launch_bounds__(kBlockThreads) void spmv_batch_kernel(const BatchJob *__restrict__ jobs,
                                                                    const int32_t *__restrict__ wave_job, int total) {
    static_assert(kWavesPerBlock == 1, "one work range per workgroup");
    using A = typename Val<VT>::A;
    const int b = xcd_block(blockIdx.x, gridDim.x, 0);  // matrices side by side: each XCD an eighth
    if (b >= total) return;
    const BatchJob &J = jobs[wave_job[b]];
    stream_range<VT, AGG, RR, LT>(J.d, b - J.wave_base, (A)J.alpha, (A)J.beta, (const A *)J.x, (A *)J.y);
}

// ---- quad kernel (natural order, spmv_kernel = 2) ---------------------------
//
// The batches are quad batches (cb_stream.h): a lane takes a quad -- four
// consecutive entries of one tile -- per pass, so the per-entry work of
// Algorithm 3 (unpack the code, multiply by the staged x, add into the row)
// runs four entries at a time.  The four codes arrive as one dword and the
// four values as one or two 16-byte loads, straight from HBM into registers
// (buffer loads on a resource covering the range's payload: an address past
// the resource reads zero instead of faulting); the LDS holds only the x
// area, the row sums, the batch's records and its tile-start marks.  A lane's
// entries that share a row are summed in a register first, so a row run costs
// one LDS add.  Pipeline per step b (one wait, at the top):
//   top       x of batch b into the x area; the panels batch b-1 finished to
//             y; batch b+2's records and tile starts into LDS
//   issue     x of batch b+1, x columns of batch b+2, records of batch b+3,
//             y of the panels batch b finishes
//   multiply  batch b from its registers
//   issue     codes and values of batch b+1 into the registers batch b freed
// A lane finds its quad's tile by one ballot of the pass's tile-start marks:
// tile = (tiles started before the pass) + (marks at or below the lane) - 1.

using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 buffer resource: 32-bit data format, no swizzle

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, int64_t bytes) {
    const uint32_t nr = bytes <= 0 ? 0u : bytes >= 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)nr, kRsrcWord3);
}

// one value at byte offset off of a buffer (0 past its end)
template <class A>
__device__ __forceinline__ A buffer_value(rsrc_t r, uint32_t off) {
    if constexpr (sizeof(A) == 8) {
        using u32x2 = unsigned int __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(A, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
    } else {
        return __builtin_bit_cast(A, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
    }
}

// raw words of one quad's four values: FP64 two 16-byte loads, FP32 one, BF16 the three aligned
// dwords around its eight bytes (BF16 values are 2-byte aligned)
template <int VS>
struct QRaw;
template <>
struct QRaw<8> {
    static constexpr int kWords = 8;
    __device__ static void load(rsrc_t r, int off, uint32_t *w) {
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, CB_TUNE_QCPOL);
        const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, CB_TUNE_QCPOL);
        w[0] = a.x, w[1] = a.y, w[2] = a.z, w[3] = a.w, w[4] = b.x, w[5] = b.y, w[6] = b.z, w[7] = b.w;
    }
};
template <>
struct QRaw<4> {
    static constexpr int kWords = 4;
    __device__ static void load(rsrc_t r, int off, uint32_t *w) {
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, CB_TUNE_QCPOL);
        w[0] = a.x, w[1] = a.y, w[2] = a.z, w[3] = a.w;
    }
};
template <>
struct QRaw<2> {
    static constexpr int kWords = 3;
    __device__ static void load(rsrc_t r, int off, uint32_t *w) {
        using u32x3 = unsigned int __attribute__((ext_vector_type(3)));
        const u32x3 a = __builtin_amdgcn_raw_buffer_load_b96(r, off & ~3, 0, CB_TUNE_QCPOL);
        w[0] = a.x, w[1] = a.y, w[2] = a.z;
    }
};
// value j of a quad from its raw words; half: the BF16 values start 2 bytes into the first word
template <int VT>
__device__ __forceinline__ typename Val<VT>::A quad_value(const uint32_t *w, int j, bool half) {
    using A = typename Val<VT>::A;
    constexpr int VS = Val<VT>::kSize;
    if constexpr (VS == 8) {
        return __hiloint2double((int)w[2 * j + 1], (int)w[2 * j]);
    } else if constexpr (VS == 4) {
        return (A)__uint_as_float(w[j]);
    } else {
        const uint32_t lo = __builtin_amdgcn_alignbit(w[1], w[0], half ? 16 : 0);
        const uint32_t hi = __builtin_amdgcn_alignbit(w[2], w[1], half ? 16 : 0);
        const uint32_t word = j < 2 ? lo : hi;
        return (A)__uint_as_float((j & 1) ? (word & 0xFFFF0000u) : (word << 16));
    }
}

// a + byte K of b, one SDWA add (written out: the compiler otherwise re-derives each byte with a
// shift and a mask from the expression that produced b)
template <int K>
__device__ __forceinline__ uint32_t add_byte(uint32_t a, uint32_t b) {
    static_assert(K >= 0 && K < 4, "a byte of a dword");
    uint32_t r;
    if constexpr (K == 0)
        asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
            : "=v"(r) : "v"(a), "v"(b));
    else if constexpr (K == 1)
        asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
            : "=v"(r) : "v"(a), "v"(b));
    else if constexpr (K == 2)
        asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2"
            : "=v"(r) : "v"(a), "v"(b));
    else
        asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3"
            : "=v"(r) : "v"(a), "v"(b));
    return r;
}
// all ones where bit j of v is set, else zero (one signed bit-field extract)
__device__ __forceinline__ int bit_mask(uint32_t v, int j) {
    int r;
    asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(r) : "v"(v), "v"(j));
    return r;
}
// v where mask is all ones, +0 where it is zero (a bitwise select, no compare)
__device__ __forceinline__ float keep_if(float v, int mask) { return __int_as_float(__float_as_int(v) & mask); }
__device__ __forceinline__ double keep_if(double v, int mask) {
    return __longlong_as_double(__double_as_longlong(v) & (long long)mask);
}

// SC: the scatter form (Algorithm 2's groups streamed): a batch's tiles come from any panels, each
// tile has accumulators of its own (slot = its position in the batch), and after the batch every
// tile's non-zero row sums are added into y with atomics (y was scaled by beta in a pre-pass).
template <int VT, int AGG, int RR, int LT, bool SC = false>
__device__ __forceinline__ void qstream_range(const DevView &d, int w, typename Val<VT>::A alpha,
                                              typename Val<VT>::A beta, const typename Val<VT>::A *__restrict__ x,
                                              typename Val<VT>::A *__restrict__ y) {
    static_assert(kWavesPerBlock == 1, "one work range per workgroup");
    static_assert(!SC || LT == 4, "the scatter form takes 16 x 16 tiles");
    static_assert(RR != 1, "the quad kernel sums a lane's row runs itself");
    static_assert(LT == 3 || LT == 4, "16 x 16 or 8 x 8 tiles");
    constexpr int S = 1 << LT;      // rows of a panel, columns of a tile
    constexpr int TPG = kWave / S;  // tiles per x gather
    constexpr int QPR = S / 4;      // quads per row of a Dense tile
    using A = typename Val<VT>::A;
    using AC = typename std::conditional<RR == 2 || RR == 4, double, A>::type;  // accumulator type
    constexpr int NACC = RR >= 3 ? 2 : 1;
    constexpr int VS = Val<VT>::kSize;
    constexpr int NWD = QRaw<VS>::kWords;
    constexpr int QT = cbs::kQTiles, QP = cbs::kQPasses;
    constexpr int NG = (QT + TPG - 1) / TPG;
    static_assert(QT % 4 == 0 && QT <= 32 && QT + 1 <= kWave, "x gathers take four tiles; records fit one load");
    constexpr int NSLOT = SC ? QT : kMaxPanels;  // accumulator slots of 16 rows
    __shared__ __align__(16) A xarea[NG * kWave];
    __shared__ __align__(16) AC acc[NSLOT * 16 * NACC];
    __shared__ __align__(16) i32x4 rtab[2][QT];
    // record word fields: the tile's first quad, and (COO/CSR) the end of its entries
    auto rec_qs = [](const i32x4 &r) { return SC ? (r.w >> 5) & 0x3FF : (r.w >> 2) & 0x3FF; };
    auto rec_lim = [](const i32x4 &r) { return SC ? (r.w >> 16) & 0x1FFF : r.z; };
    __shared__ __align__(16) uint32_t marks[2][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    if (w >= d.nwaves) return;
    const int o_begin = d.batch_ptr[w], o_end = d.batch_ptr[w + 1];
    if (o_begin >= o_end) return;
    const int oend = o_end - o_begin;
    const int t0 = d.wave_ptr[w], t1 = d.wave_ptr[w + 1];
    const int64_t pbase = d.tile_vp[t0];
    const rsrc_t prs = make_rsrc(d.payload + pbase, d.payload_alloc - pbase);
    const rsrc_t rrs = make_rsrc(d.batch_stream + 4 * (int64_t)o_begin, d.stream_alloc - 16 * (int64_t)o_begin);
    const int p_first = d.tile_row[t0], p_last = d.tile_row[t1 - 1];
    const bool sh_first = d.panel_shared[p_first] != 0, sh_last = d.panel_shared[p_last] != 0;
    const int gj = lane >> LT, glc = lane & (S - 1);

    // header and records of the batch at record o (relative to the range's first): lane 63 the
    // header, lane i < QT record i (lanes QT .. 62 record QT - 1 again)
    i32x4 Q;
    auto qload = [&](int o) {
        const int r = lane == kWave - 1 ? o : o + 1 + min(lane, QT - 1);
        Q = __builtin_bit_cast(i32x4, __builtin_amdgcn_raw_buffer_load_b128(rrs, 16 * r, 0, CB_TUNE_QCPOL));
    };
    struct Hdr {
        int pb, nt, np, done, qtot, cbase;
    };
    auto header = [&]() {
        const int hz = __builtin_amdgcn_readlane(Q.y, kWave - 1);
        return Hdr{__builtin_amdgcn_readlane(Q.x, kWave - 1), hz & 0xFF, (hz >> 8) & 0xFF, (hz >> 16) & 0xF,
                   __builtin_amdgcn_readlane(Q.z, kWave - 1), AGG == 3 ? __builtin_amdgcn_readlane(Q.w, kWave - 1) : 0};
    };
    // the records in Q (header h) into record table `par`, and the tiles' first quads as marks: byte
    // (p, l) of the mark table is set where tile starts at quad 64 p + l
    auto stage = [&](const Hdr &h, int par) {
        marks[par][lane] = 0u;
        if (lane < h.nt) {
            rtab[par][lane] = Q;
            const int qs = rec_qs(Q);
            reinterpret_cast<uint8_t *>(marks[par])[4 * (qs & 63) + ((qs >> 6) & 3)] = 1;
        }
    };

    // x of a batch whose first tile is tb (nt tiles), as in the streaming kernel.  The tile columns
    // and x are read through buffer resources: the range's tile columns (a load past the range's
    // last tile returns 0, a valid column) and x (n below 2^29, so every column's byte offset fits
    // 32 bits; a load past column n - 1 returns 0).  One offset per batch, a constant per gather.
    // Compressed columns: 2-byte offsets through a resource over the range's tiles, plus (AGG 2) each
    // tile's 4-byte base through another (past the range's last tile both read 0: column 0) or
    // (AGG 3) the batch's base from its header (past the last tile: the batch's lowest column)
    constexpr bool C16 = AGG >= 2;
    constexpr int CW = C16 ? 2 * S : AGG ? 4 * S : 4;  // bytes of tile columns per tile
    const rsrc_t crs = C16 ? make_rsrc(d.tile_c16 + S * (int64_t)t0, CW * (int64_t)(t1 - t0))
                       : AGG    ? make_rsrc(d.tile_cols + S * (int64_t)t0, CW * (int64_t)(t1 - t0))
                                : make_rsrc(d.tile_col + t0, CW * (int64_t)(t1 - t0));
    const rsrc_t brs = make_rsrc(AGG == 2 ? d.tile_cbase + t0 : d.tile_col, 4 * (int64_t)(t1 - t0));
    const rsrc_t xrs = make_rsrc(x, d.n * (int64_t)sizeof(A));
    const int cl = C16 ? 2 * (S * gj + glc) : AGG ? 4 * (S * gj + (glc & 3) * (S / 4) + (glc >> 2)) : 4 * gj;
    int RG[NG];
    int RB[AGG == 2 ? NG : 1];
    auto issue_cols = [&](int tb, int nt) {
        const int cb0 = CW * (tb - t0) + cl;
#pragma unroll
        for (int g = 0; g < NG; ++g)
            if (TPG * g < nt) {
                if constexpr (C16) {
                    RG[g] = (int)__builtin_amdgcn_raw_buffer_load_b16(crs, cb0 + CW * TPG * g, 0, CB_TUNE_QCPOL);
                    if constexpr (AGG == 2)
                        RB[g] = (int)__builtin_amdgcn_raw_buffer_load_b32(brs, 4 * (tb - t0 + TPG * g + gj), 0,
                                                                           CB_TUNE_QCPOL);
                } else {
                    RG[g] = (int)__builtin_amdgcn_raw_buffer_load_b32(crs, cb0 + CW * TPG * g, 0, CB_TUNE_QCPOL);
                }
            }
    };
    A XG[NG];
    auto issue_x = [&](const Hdr &h) {
#pragma unroll
        for (int g = 0; g < NG; ++g)
            if (TPG * g < h.nt) {
                uint32_t col;
                if constexpr (AGG == 3) col = (uint32_t)(RG[g] + h.cbase);
                else if constexpr (AGG == 2) col = (uint32_t)(RG[g] + RB[g]);
                else col = (uint32_t)RG[g] * (AGG ? 1u : (uint32_t)S) + (AGG ? 0u : (uint32_t)glc);
                XG[g] = buffer_value<A>(xrs, col * (uint32_t)sizeof(A));
            }
    };
    auto put_x = [&](int nt) {
#pragma unroll
        for (int g = 0; g < NG; ++g)
            if (TPG * g < nt) xarea[64 * g + lane] = XG[g];
    };

    // the quads of a batch in flight: codes, value words and a word of what the multiply needs
    //   bits 0-8 x-area index of the tile, 9-15 accumulator offset (slot, copy), 16 Dense,
    //   17-20 the entries present (COO/CSR) or 17-24 the first code and 25-27 the bitmap nibble
    //   (Dense), 31 BF16 values start 2 bytes into their first word
    uint32_t C[QP], M[QP], W[QP][NWD];
    auto issue_payload = [&](const Hdr &h, int par) {
        const uint32_t mk = marks[par][lane];
        int jb = 0;
#pragma unroll
        for (int p = 0; p < QP; ++p) {
            if (p < h.np) {
                const uint64_t bal = __builtin_amdgcn_ballot_w64(((mk >> (8 * p)) & 0xFFu) != 0u);
                const int below =
                    (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                const int ti = jb + below + (int)((bal >> lane) & 1u) - 1;
                jb += __builtin_popcountll(bal);
                const i32x4 r = rtab[par][max(ti, 0)];
                const int q = 64 * p + lane;
                const bool live = q < h.qtot;
                const bool dense = live && ((r.w >> 15) & 1);
                // scatter form: the slot is the tile's position, taken from the x-area index in multiply
                const int slot = SC ? 0 : r.w & (kMaxPanels - 1);
                uint32_t m = (uint32_t)(ti << LT) |
                             ((uint32_t)(slot * 16 * NACC + (NACC == 2 ? (lane & 1) << 4 : 0)) << 9);
                int caddr;
                if (dense) {
                    // quad dq of a Dense tile: row dq / QPR, columns 4 (dq mod QPR) .. + 3, i.e. elements
                    // 4 dq .. 4 dq + 3 of the row-major tile and bits 4 dq .. of its bitmap
                    const int dq = q - rec_qs(r);
                    caddr = r.x + 4 * (dq >> 3);
                    m |= (1u << 16) | ((uint32_t)(((dq % QPR) << 6) | (dq / QPR)) << 17) | ((uint32_t)(dq & 7) << 25);
                } else {
                    const int nv = live ? min(max(rec_lim(r) - 4 * q, 0), 4) : 0;
                    caddr = r.x + 4 * q;
                    m |= (uint32_t)((1 << nv) - 1) << 17;
                }
                const int vaddr = r.y + 4 * VS * q;
                if (VS == 2) m |= (uint32_t)(vaddr & 2) << 30;
                M[p] = m;
                C[p] = __builtin_amdgcn_raw_buffer_load_b32(prs, caddr, 0, CB_TUNE_QCPOL);
                QRaw<VS>::load(prs, vaddr, W[p]);
            }
        }
    };
    auto multiply = [&](int np) {
#pragma unroll
        for (int p = 0; p < QP; ++p) {
            if (p < np) {
                const uint32_t m = M[p];
                uint32_t codes, vm;
                if ((m >> 16) & 1u) {
                    vm = (C[p] >> (4 * ((m >> 25) & 7u))) & 0xFu;
                    codes = ((m >> 17) & 0xFFu) * 0x01010101u + 0x30201000u;
                } else {
                    vm = (m >> 17) & 0xFu;
                    codes = C[p];
                }
                const int xo = (int)(m & 0x1FFu);
                const int ao = SC ? (xo >> LT) * 16 * NACC + (NACC == 2 ? (lane & 1) << 4 : 0) : (int)((m >> 9) & 0x7Fu);
                const bool half = (m >> 31) != 0u;
                // the four x reads issued together: a code's column nibble, masked to the tile's width,
                // names one of the tile's x slots, so an absent entry's read stays inside the x area.
                // xb: each entry's x slot as a byte offset from the tile's first, one byte per entry
                constexpr int XSH = sizeof(A) == 8 ? 3 : 2;
                const uint32_t xb = (codes >> (4 - XSH)) & (0x01010101u * (uint32_t)((S - 1) << XSH));
                const uint32_t x0 = (uint32_t)xo << XSH;
                const char *xa = reinterpret_cast<const char *>(xarea);
                A xq[4];
                xq[0] = *reinterpret_cast<const A *>(xa + add_byte<0>(x0, xb));
                xq[1] = *reinterpret_cast<const A *>(xa + add_byte<1>(x0, xb));
                xq[2] = *reinterpret_cast<const A *>(xa + add_byte<2>(x0, xb));
                xq[3] = *reinterpret_cast<const A *>(xa + add_byte<3>(x0, xb));
                // rb: each entry's row accumulator as a byte offset from the slot's first
                constexpr int ASH = sizeof(AC) == 8 ? 3 : 2;
                const uint32_t rb = (codes << ASH) & (0x01010101u * (uint32_t)(15 << ASH));
                const uint32_t a0 = (uint32_t)ao << ASH;
                char *aa = reinterpret_cast<char *>(acc);
                AC s = AC(0);
                uint32_t run = add_byte<0>(a0, rb);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t row = j == 0 ? run : j == 1 ? add_byte<1>(a0, rb) : j == 2 ? add_byte<2>(a0, rb)
                                                                                              : add_byte<3>(a0, rb);
                    // an absent entry adds a zero product.  With FP32 and BF16 values it also keeps the
                    // current run.  With FP64 values (registers at their limit) it takes whatever row
                    // its code byte names: absent entries only follow the present ones of a COO or CSR
                    // tile (or sit in a Dense quad, whose four entries share one row), and every row
                    // nibble names one of the slot's accumulators, so such a switch only adds zeros
                    const int okm = bit_mask(vm, j);
                    const A prod = keep_if(quad_value<VT>(W[p], j, half) * xq[j], okm);
                    const uint32_t rk = VS == 8 ? row : (row & (uint32_t)okm) | (run & ~(uint32_t)okm);
                    if (rk != run) {
                        lds_add(reinterpret_cast<AC *>(aa + run), s);
                        s = AC(0);
                        run = rk;
                    }
                    s += (AC)prod;
                }
                if (vm) lds_add(reinterpret_cast<AC *>(aa + run), s);
            }
        }
    };

    // panels finished by a batch, as in the streaming kernel
    const int fk = lane >> 4, fr = lane & 15;
    A YP = A(0);
    int done_pb = 0, done_mask = 0;
    auto is_shared = [&](int p) { return (p == p_first && sh_first) || (p == p_last && sh_last); };
    auto issue_y = [&]() {
        if (beta == A(0)) return;
        const int64_t row = S * (int64_t)(done_pb + fk) + fr;
        if (((done_mask >> fk) & 1) && fr < S && row < d.m && !is_shared(done_pb + fk)) YP = y[row];
    };
    auto flush = [&]() {
        if ((done_mask >> fk) & 1) {
            const int p = done_pb + fk;
            AC *a = &acc[(p & (kMaxPanels - 1)) * 16 * NACC + fr];
            AC sv = *a;
            *a = AC(0);
            if constexpr (NACC == 2) {
                sv += a[16];
                a[16] = AC(0);
            }
            const A v = (A)sv;
            const int64_t row = S * (int64_t)p + fr;
            if (fr < S && row < d.m) {
                if (is_shared(p)) {
                    global_add(&y[row], alpha * v);
                } else {
                    A r = alpha * v;
                    if (beta != A(0)) r += beta * YP;
                    y[row] = r;
                }
            }
        }
        done_mask = 0;
    };

    for (int i = lane; i < NSLOT * 16 * NACC; i += kWave) acc[i] = AC(0);
    // scatter form: the panels of the batch being multiplied, lane (fk, fr) for its tiles fk + 4 j
    int PN[4] = {0, 0, 0, 0};
    auto scatter_panels = [&](const Hdr &h, int par) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (fk + 4 * j < h.nt) PN[j] = rtab[par][fk + 4 * j].z;
    };
    // scatter form: every tile's row sums of the batch just multiplied added into y
    auto scatter_flush = [&](int nt) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int t = fk + 4 * j;
            if (t < nt) {
                AC *a = &acc[t * 16 * NACC + fr];
                AC sv = *a;
                *a = AC(0);
                if constexpr (NACC == 2) {
                    sv += a[16];
                    a[16] = AC(0);
                }
                const int64_t row = 16 * (int64_t)PN[j] + fr;
                if (sv != AC(0) && row < d.m) global_add(&y[row], alpha * (A)sv);
            }
        }
    };
    // prologue: batch 0's records, x columns, payload and x; batch 1's records and x columns; batch
    // 2's records in flight.  At the top of step b the registers hold the payload and x of batch b,
    // the x columns of batch b+1 and Q the records of batch b+2; the tables hold batches b and b+1.
    qload(0);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    Hdr h0 = header(), h1{}, h2{};
    stage(h0, 0);
    issue_cols(t0, h0.nt);
    int o1 = 1 + h0.nt;
    const int tb1 = t0 + h0.nt;
    if (o1 < oend) qload(o1);
    __builtin_amdgcn_wave_barrier();
    issue_payload(h0, 0);
    issue_x(h0);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    int o2 = o1, tb2 = tb1;
    if (o1 < oend) {
        h1 = header();
        stage(h1, 1);
        issue_cols(tb1, h1.nt);
        o2 = o1 + 1 + h1.nt;
        tb2 = tb1 + h1.nt;
        if (o2 < oend) qload(o2);
    }
    int par = 0;  // record table of batch b
    int ob = 0;
    while (ob < oend) {
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        put_x(h0.nt);
        if constexpr (SC) scatter_panels(h0, par);
        else flush();
        const bool have1 = o1 < oend, have2 = o2 < oend;
        int o3 = o2;
        if (have2) {
            h2 = header();
            stage(h2, par);  // batch b+2 takes batch b's table (batch b's payload was issued a step ago)
        }
        __builtin_amdgcn_wave_barrier();
        if (have1) issue_x(h1);
        if (have2) o3 = o2 + 1 + h2.nt;
        if constexpr (!SC) {
            done_pb = h0.pb;
            done_mask = h0.done;
            issue_y();
        }
        multiply(h0.np);
        if constexpr (SC) scatter_flush(h0.nt);
        __builtin_amdgcn_wave_barrier();
        // issued after the multiply, so their registers are free while it runs; they are waited for
        // at the top of the next step with the payload
        if (have1) issue_payload(h1, par ^ 1);
        if (have2) {
            issue_cols(tb2, h2.nt);
            if (o3 < oend) qload(o3);
        }
        ob = o1;
        h0 = h1;
        o1 = o2;
        h1 = h2;
        o2 = o3;
        tb2 += have2 ? h2.nt : 0;
        par ^= 1;
    }
    if constexpr (!SC) flush();
}

// The serving loop's batched launch for quad-batch structures (as spmv_batch_kernel)
template <int VT, int AGG, int RR, int LT>
__global__ __launch_bounds__(kBlockThreads) void spmv_qbatch_kernel(const BatchJob *__restrict__ jobs,
                                                                     const int32_t *__restrict__ wave_job, int total) {
    using A = typename Val<VT>::A;
    const int b = xcd_block(blockIdx.x, gridDim.x, 0);  // matrices side by side: each XCD an eighth
    if (b >= total) return;
    const BatchJob &J = jobs[wave_job[b]];
    qstream_range<VT, AGG, RR, LT>(J.d, b - J.wave_base, (A)J.alpha, (A)J.beta, (const A *)J.x, (A *)J.y);
}

#ifndef CB_TUNE_QWAVES
#define CB_TUNE_QWAVES 6  // natural-order quad kernel: at least this many wavefronts per SIMD (register cap)
#endif
#ifndef CB_TUNE_QWAVES_C16
#define CB_TUNE_QWAVES_C16 5  // the same for FP64 values with 2-byte column offsets (one more register per gather)
#endif
template <int VT, int AGG, int RR, int LT, bool SC>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(SC ? 1 : (AGG == 2 && VT == 0) ? CB_TUNE_QWAVES_C16 : CB_TUNE_QWAVES))) void spmv_quad_kernel(DevView d, typename Val<VT>::A alpha,
                                                                   typename Val<VT>::A beta,
                                                                   const typename Val<VT>::A *__restrict__ x,
                                                                   typename Val<VT>::A *__restrict__ y) {
    qstream_range<VT, AGG, RR, LT, SC>(d, xcd_block(blockIdx.x, gridDim.x, d.xcd_chunk), alpha, beta, x, y);
}

// ---- rows per lane (natural order) -----------------------------------------
//
// Each 16-lane group of the wavefront takes every fourth panel of the work range and walks the
// panel's tiles; lane r of the group owns row r of the panel and keeps its sum in a register.  CSR
// tiles: lane r multiplies the entries of row r (the tile's one-byte row starts give them);
// COO tiles: lanes take entries r, r + 16, ... and add their products into the group's 16 row sums
// in LDS; Dense tiles: lane r takes row r's 16 values, occupancy bits honoured.  The group gathers a
// tile's 16 x values (lane c takes column c) into its LDS x area; the next tile's record and column
// are loaded while the current tile is multiplied.  Sums are kept in FP64.
template <int VT, bool AGG>
__global__ __launch_bounds__(kBlockThreads) void spmv_rows_kernel(DevView d, typename Val<VT>::A alpha,
                                                                   typename Val<VT>::A beta,
                                                                   const typename Val<VT>::A *__restrict__ x,
                                                                   typename Val<VT>::A *__restrict__ y) {
    static_assert(kWavesPerBlock == 1, "one wavefront per workgroup");
    using A = typename Val<VT>::A;
    constexpr int VS = Val<VT>::kSize;
    __shared__ double gacc[4][16];
    __shared__ A xs[4][16];
    const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, r = lane & 15;
    const int w = xcd_block(blockIdx.x, gridDim.x, d.xcd_chunk);
    if (w >= d.nwaves) return;
    const int t0 = d.wave_ptr[w], t1 = d.wave_ptr[w + 1];
    if (t0 >= t1) return;
    const int p_first = d.tile_row[t0], p_last = d.tile_row[t1 - 1];
    const bool sh_first = d.panel_shared[p_first] != 0, sh_last = d.panel_shared[p_last] != 0;
    const i32x4 *recs = reinterpret_cast<const i32x4 *>(d.tile_rec);
    gacc[g][r] = 0.0;
    // column of lane r in tile t: tile_cols holds column c at position (c mod 4) * 4 + c / 4
    auto column = [&](int t, int cb) -> int {
        if (AGG) return d.tile_cols[16 * (size_t)t + (r & 3) * 4 + (r >> 2)];
        const int64_t c = 16 * (int64_t)cb + r;
        return c < d.n ? (int)c : 0;
    };
    for (int p = p_first + g; p <= p_last; p += 4) {
        const int tb = max(d.panel_tile[p], t0), te = min(d.panel_tile[p + 1], t1);
        double acc = 0.0;
        i32x4 rec_n = recs[min(tb, t1 - 1)];
        int col_n = column(min(tb, t1 - 1), rec_n.w);
        for (int t = tb; t < te; ++t) {
            const i32x4 rec = rec_n;
            const int col = col_n;
            if (t + 1 < te) {
                rec_n = recs[t + 1];
                col_n = column(t + 1, rec_n.w);
            }
            const A xv = x[col];
            const uint64_t vp = (uint64_t)(uint32_t)rec.x | ((uint64_t)((uint32_t)rec.y & 0xFFFFu) << 32);
            const int type = ((uint32_t)rec.y >> 16) & 3, nnz = (int)((uint32_t)rec.y >> 18) + 1;
            const uint8_t *base = d.payload + vp;
            xs[g][r] = xv;
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the group's x values are in LDS
            __builtin_amdgcn_wave_barrier();
            if (type == 1) {
                // CSR: row starts, codes, values
                const int s0 = base[r], s1 = r < 15 ? (int)base[r + 1] : nnz;
                const uint8_t *codes = base + 16;
                const uint8_t *vals = codes + nnz + pad_bytes(16 + nnz, VS);
                int e = s0;
                for (; e + 1 < s1; e += 2) {
                    const uint32_t c0 = codes[e], c1 = codes[e + 1];
                    const A v0 = Val<VT>::load(vals, e), v1 = Val<VT>::load(vals, e + 1);
                    acc += (double)v0 * (double)xs[g][c0 >> 4];
                    acc += (double)v1 * (double)xs[g][c1 >> 4];
                }
                if (e < s1) acc += (double)Val<VT>::load(vals, e) * (double)xs[g][codes[e] >> 4];
            } else if (type == 0) {
                // COO: codes, values; entries r, r + 16, ...
                const uint8_t *vals = base + nnz + pad_bytes(nnz, VS);
                for (int e = r; e < nnz; e += 16) {
                    const uint32_t c = base[e];
                    const double prod = (double)Val<VT>::load(vals, e) * (double)xs[g][c >> 4];
                    __hip_atomic_fetch_add(&gacc[g][c & 15], prod, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                }
            } else {
                // Dense: 256 values, then the 32-byte occupancy bitmap
                const uint32_t bits = (uint32_t)base[256 * VS + 2 * r] | ((uint32_t)base[256 * VS + 2 * r + 1] << 8);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    A v[4];
                    Val<VT>::load4(base, 16 * r + 4 * q, v);
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if ((bits >> (4 * q + j)) & 1u) acc += (double)v[j] * (double)xs[g][4 * q + j];
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        // the panel's row sums: registers plus the COO contributions in LDS
        __builtin_amdgcn_s_waitcnt(0xC07F);
        acc += gacc[g][r];
        gacc[g][r] = 0.0;
        const int64_t row = 16 * (int64_t)p + r;
        if (tb < te && row < d.m) {
            const A v = (A)acc;
            if ((p == p_first && sh_first) || (p == p_last && sh_last)) {
                global_add(&y[row], alpha * v);
            } else {
                A out = alpha * v;
                if (beta != A(0)) out += beta * y[row];
                y[row] = out;
            }
        }
    }
}

// ---- k right-hand sides ---------------------------------------------------
//
// Y = alpha*A*X + beta*Y with X (n x k) and Y (m x k) row-major.  A launch
// slice (blockIdx.y) covers KC columns of X.  A wavefront walks its tiles as
// spmv_kernel does; lane (r, q) owns row r of the current panel and KC/4
// consecutive columns, in registers.  Per tile the X rows of the tile's 16
// columns are staged in LDS; each lane walks the entries of its row (row
// starts from the CSR header, or counted with ballots for COO tiles) and
// updates its KC/4 accumulators.  Dense tiles are multiplied on the matrix
// cores: the 16x16 tile times the 16 x KC block of X as 16x16x4 MFMA steps
// (FP64 values: v_mfma_f64_16x16x4_f64; FP32/BF16 values: v_mfma_f32_16x16x4_f32),
// unless one of the staged X values is Inf or NaN, where the zero fill of the
// tile would contribute 0*Inf; those tiles take the entry-by-entry path.

// packed region size of a tile (16-byte aligned), as laid out by the converter
// bytes of a tile's packed region (S = 1 << lt), rounded to the 16-byte tile alignment
template <int VS>
__device__ __forceinline__ int region_dev(int ty, int nz, int lt) {
    const int S = 1 << lt;
    int b;
    if (ty == 0)
        b = nz + pad_bytes(nz, VS) + nz * VS;
    else if (ty == 1)
        b = S + nz + pad_bytes(S + nz, VS) + nz * VS;
    else
        b = S * S * VS + S * S / 8;
    return (b + 15) & ~15;
}

template <class A>
struct Mfma;
// Operands of both shapes: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16].  The
// accumulator differs: element v of lane l is D[4v + l/16][l % 16] for FP64 and
// D[4(l/16) + v][l % 16] for FP32 (checked on gfx950 with one-hot operands).
template <>
struct Mfma<double> {
    using C = double __attribute__((ext_vector_type(4)));
    __device__ static C step(double a, double b, C c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <>
struct Mfma<float> {
    using C = float __attribute__((ext_vector_type(4)));
    __device__ static C step(float a, float b, C c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <int VT, int KC>
__global__ __launch_bounds__(kBlockThreads) void spmm_kernel(DevView d, typename Val<VT>::A alpha,
                                                              typename Val<VT>::A beta,
                                                              const typename Val<VT>::A *__restrict__ X, int64_t ldx,
                                                              typename Val<VT>::A *__restrict__ Y, int64_t ldy,
                                                              int k) {
    // One-tile software pipeline.  While tile t is multiplied out of LDS, the
    // loads of tile t+1 (its packed region, three 1 KB wave loads, and its 16 X
    // rows) and the restore_cols entries of tile t+2 are in flight; the scalar
    // metadata of tile t+2 is read through the scalar cache.
    using A = typename Val<VT>::A;
    constexpr int VS = Val<VT>::kSize;
    constexpr int NJ = KC / 4;  // columns per lane
    __shared__ __align__(16) uint8_t tbuf_all[kWavesPerBlock][3 * kChunk];
    __shared__ A xs_all[kWavesPerBlock][16 * KC];
    __shared__ A cs_all[kWavesPerBlock][KC >= 16 ? 16 * KC : 1];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int w = xcd_block(blockIdx.x, gridDim.x, d.xcd_chunk) * kWavesPerBlock + wid;
    if (w >= d.nwaves) return;
    const int j0 = blockIdx.y * KC;
    const int kc = min(KC, k - j0);
    uint8_t *tbuf = tbuf_all[wid];
    A *xs = xs_all[wid];
    A *cs = cs_all[wid];
    const int t0 = d.wave_ptr[w], t1 = d.wave_ptr[w + 1];
    // lane (r4, q4) owns row r4 of the panel (rows past the tile size S idle) and KC/4 columns of Y
    const int r4 = lane >> 2, q4 = lane & 3, jb = q4 * NJ;
    const int LT = d.tile_lt, TS = 1 << LT;
    A acc[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) acc[i] = A(0);

    auto flush = [&](int p, bool shared) {
        const int64_t row = ((int64_t)p << LT) + r4;
        if (r4 < TS && row < d.m) {
            A *yp = Y + row * ldy + j0 + jb;
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                if (jb + i < kc) {
                    if (shared) {
                        global_add(&yp[i], alpha * acc[i]);
                    } else {
                        A out = alpha * acc[i];
                        if (beta != A(0)) out += beta * yp[i];
                        yp[i] = out;
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < NJ; ++i) acc[i] = A(0);
    };

    // per-tile scalar metadata
    struct TM {
        int row, col, nts;  // nts = nz | type << 16 | panel-shared << 24
        int64_t vp;
    };
    auto meta = [&](int t) {
        TM m;
        const int tc = min(t, t1 - 1);
        m.row = d.tile_row[tc];
        m.col = d.tile_col[tc];
        m.vp = d.tile_vp[tc];
        // the panel flag is read two tiles ahead of its use at the panel's flush
        m.nts = d.tile_nnz[tc] | (uniform_byte(d.tile_type, tc) << 16) | (uniform_byte(d.panel_shared, m.row) << 24);
        return m;
    };
    // original column of local column r4 of a tile (restore entry read one tile ahead)
    auto restore_entry = [&](const TM &m) {
        if (!d.col_agg) return 0;
        const int a = d.cols_offset[m.row] + (m.col << LT) + r4;
        return d.restore_cols[min(a, d.cols_offset[m.row + 1] - 1)];
    };
    auto colvalid = [&](const TM &m) {
        if (r4 >= TS) return false;
        if (d.col_agg) return d.cols_offset[m.row] + (m.col << LT) + r4 < d.cols_offset[m.row + 1];
        return ((int64_t)m.col << LT) + r4 < d.n;
    };
    // loads of one tile: its packed region (chunks past the region end re-read the last one) and
    // its X rows (lane (r4, q4): column r4, KC/4 entries; columns outside the tile read row 0)
    u32x4 P[3];
    A XR[NJ];
    auto issue_tile = [&](const TM &m, int rcol, bool cv) {
        const int last = (region_dev<VS>((m.nts >> 16) & 0xFF, m.nts & 0xFFFF, LT) - 1) >> 10;
        const u32x4 *src = reinterpret_cast<const u32x4 *>(d.payload + m.vp) + lane;
#pragma unroll
        for (int i = 0; i < 3; ++i) P[i] = src[min(i, last) * kWave];
        const int64_t col = d.col_agg ? rcol : ((int64_t)m.col << LT) + r4;
        const int64_t rowoff = cv ? col * ldx : 0;
#pragma unroll
        for (int i = 0; i < NJ; ++i) XR[i] = X[rowoff + j0 + min(jb + i, kc - 1)];
    };

    // prologue: tile t0's loads, tile t0+1's restore entry
    TM m_cur = meta(t0);
    TM m_nxt = meta(t0 + 1);
    issue_tile(m_cur, restore_entry(m_cur), colvalid(m_cur));
    int rc_nxt = restore_entry(m_nxt);
    int cur = -1, cur_sh = 0;
    for (int t = t0; t < t1; ++t) {
        // 1. tile t's data into LDS
        const bool cv = colvalid(m_cur);
#pragma unroll
        for (int i = 0; i < 3; ++i) reinterpret_cast<u32x4 *>(tbuf)[i * kWave + lane] = P[i];
        // columns past kc hold a clamped copy; their sums are never written back
        bool finite = true;
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            const A xv = cv ? XR[i] : A(0);
            finite = finite && __builtin_isfinite(xv);
            xs[r4 * KC + jb + i] = xv;
        }
        // 2. tile t+1's loads and tile t+2's restore entry and metadata
        const TM m = m_cur;
        const TM m2 = meta(t + 2);
        issue_tile(m_nxt, rc_nxt, colvalid(m_nxt));
        rc_nxt = restore_entry(m2);
        m_cur = m_nxt;
        m_nxt = m2;
        // 3. tile t
        if (m.row != cur) {
            if (cur >= 0) flush(cur, cur_sh != 0);
            cur = m.row;
            cur_sh = m.nts >> 24;
        }
        const int nz = m.nts & 0xFFFF, ty = (m.nts >> 16) & 0xFF;
        if (ty == 2 && KC >= 16 && TS == 16 && __ballot(!finite) == 0) {
            // dense tile on the matrix cores: C(16 x 16 block ob) = sum_kb D[:, 4kb:4kb+4] X[4kb:4kb+4, block]
            const int li = lane & 15, lk = lane >> 4;
            A a[4];
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) a[kb] = Val<VT>::load(tbuf, li * 16 + 4 * kb + lk);
#pragma unroll
            for (int ob = 0; ob < KC / 16; ++ob) {
                typename Mfma<A>::C cvec = {A(0), A(0), A(0), A(0)};
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) cvec = Mfma<A>::step(a[kb], xs[(4 * kb + lk) * KC + ob * 16 + li], cvec);
#pragma unroll
                for (int v = 0; v < 4; ++v) cs[Mfma<A>::row(lane, v) * KC + ob * 16 + li] = cvec[v];
            }
#pragma unroll
            for (int i = 0; i < NJ; ++i) acc[i] += cs[r4 * KC + jb + i];
            continue;
        }
        if (ty == 2) {
            // entry by entry over the occupancy bitmap of row r4 (bits r4 S .. r4 S + S - 1)
            const uint8_t *mask = tbuf + TS * TS * VS;
            const int eb = (r4 * TS) >> 3;
            const uint32_t bits =
                r4 < TS ? ((uint32_t)mask[eb] | ((uint32_t)mask[eb + 1] << 8)) & ((1u << TS) - 1u) : 0u;
            for (int cc = 0; cc < TS; ++cc) {
                if ((bits >> cc) & 1u) {
                    const A v = Val<VT>::load(tbuf, r4 * TS + cc);
#pragma unroll
                    for (int i = 0; i < NJ; ++i) acc[i] += v * xs[cc * KC + jb + i];
                }
            }
            continue;
        }
        const int hdr = ty == 1 ? TS : 0;
        const uint8_t *codes = tbuf + hdr;
        const uint8_t *vals = codes + nz + pad_bytes(hdr + nz, VS);
        int rs, re;
        if (ty == 1) {
            rs = r4 < TS ? (int)tbuf[r4] : 0;
            re = r4 < TS - 1 ? (int)tbuf[r4 + 1] : r4 == TS - 1 ? nz : 0;
        } else {
            // COO: entries are row-major; row r4 spans the entries with row < r4 + 1 minus those with row < r4
            rs = 0;
            re = 0;
            for (int e0 = 0; e0 < nz; e0 += kWave) {
                const int e = e0 + lane;
                const int row_e = e < nz ? (int)(codes[e] & 15) : 16;
#pragma unroll
                for (int r = 1; r <= 16; ++r) {
                    const int cnt = __popcll(__ballot(row_e < r));
                    if (r == r4) rs += cnt;
                    if (r == r4 + 1) re += cnt;
                }
            }
        }
        for (int e = rs; e < re; ++e) {
            const A v = Val<VT>::load(vals, e);
            const int lc = codes[e] >> 4;
#pragma unroll
            for (int i = 0; i < NJ; ++i) acc[i] += v * xs[lc * KC + jb + i];
        }
    }
    if (cur >= 0) flush(cur, cur_sh != 0);
}

// y <- beta * y (0 when beta == 0) on the rows of shared and empty panels (panels of 1 << lt rows)
template <class A>
__global__ void prepass_kernel(const int32_t *__restrict__ list, int32_t np, int64_t m, A beta, A *__restrict__ y,
                               int k, int64_t ldy, int lt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = ((int64_t)k) << lt;
    if (i >= (int64_t)np * per) return;
    const int64_t pi = i / per, rem = i - pi * per;
    const int64_t row = ((int64_t)list[pi] << lt) + rem / k;
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

// Each wavefront reads its own contiguous 16 KB span (as a product's wavefront reads its range),
// four 16-byte loads in flight per lane with the nontemporal hint, folded into one word; the store
// happens only when the fold equals a fixed value, which keeps every load.  Measured the fastest
// read pattern on gfx950 (1 GiB: 6.93 TB/s; without the hint 6.19, with eight loads in flight or
// 64 KB spans 5.8-5.9; grid-stride loops reach about 10 % less).
constexpr int64_t kReadSpan16 = 1024;  // 16-byte units per wavefront
__global__ __launch_bounds__(256) void read_kernel(const uint4 *__restrict__ src, int64_t n16,
                                                   uint4 *__restrict__ sink) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    const int64_t end = min(w * kReadSpan16 + kReadSpan16, n16);
    int64_t i = w * kReadSpan16 + lane;
    uint32_t f = 0;
    const u32x4 *s4 = reinterpret_cast<const u32x4 *>(src);
    for (; i + 3 * kWave < end; i += 4 * kWave) {
        const u32x4 a = ld_stream<true>(s4 + i), b = ld_stream<true>(s4 + i + kWave),
                    c = ld_stream<true>(s4 + i + 2 * kWave), e = ld_stream<true>(s4 + i + 3 * kWave);
        f ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ e.x ^ e.y ^ e.z ^ e.w;
    }
    for (; i < end; i += kWave) {
        const u32x4 a = ld_stream<true>(s4 + i);
        f ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    if (f == 0x9E3779B9u) sink[0] = make_uint4(f, f, f, f);
}

template <class A>
hipError_t prepass(const DevView &d, double beta, void *y, int k, int64_t ldy, hipStream_t s) {
    if (d.nprepass <= 0) return hipSuccess;
    const int64_t total = ((int64_t)d.nprepass * k) << d.tile_lt;
    const int64_t nb = (total + 255) / 256;
    hipLaunchKernelGGL(prepass_kernel<A>, dim3((unsigned)nb), dim3(256), 0, s, d.prepass_list, d.nprepass, d.m,
                       (A)beta, (A *)y, k, ldy, (int)d.tile_lt);
    return hipGetLastError();
}

// the natural-order kernels of one value type and tile size, chosen by aggregation and row-sum mode
// (FP64 accumulators already: modes 2 and 4 are modes 0 and 3)
template <int VT, int LT>
hipError_t spmv_stream_launch(const DevView &d, typename Val<VT>::A a, typename Val<VT>::A b, const void *x, void *y,
                              int nb, hipStream_t s) {
    using A = typename Val<VT>::A;
    constexpr bool kWide = std::is_same<A, double>::value;
    constexpr int kRR2 = kWide ? 0 : 2, kRR4 = kWide ? 3 : 4;
    const int rr = d.row_reduce;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlockThreads), 0, s, d, a, b, (const A *)x, (A *)y);
    };
    auto by_rr = [&](auto agg) {
        constexpr int AG = decltype(agg)::value;
        if (rr == 1) go(spmv_stream_kernel<VT, AG, 1, LT>);
        else if (rr == 2) go(spmv_stream_kernel<VT, AG, kRR2, LT>);
        else if (rr == 3) go(spmv_stream_kernel<VT, AG, 3, LT>);
        else if (rr == 4) go(spmv_stream_kernel<VT, AG, kRR4, LT>);
        else go(spmv_stream_kernel<VT, AG, 0, LT>);
    };
    if (d.col_agg == 2) by_rr(std::integral_constant<int, 2>());
    else if (d.col_agg) by_rr(std::integral_constant<int, 1>());
    else by_rr(std::integral_constant<int, 0>());
    return hipGetLastError();
}

template <int VT, int LT, bool SC = false>
hipError_t spmv_quad_launch(const DevView &d, typename Val<VT>::A a, typename Val<VT>::A b, const void *x, void *y,
                            int nb, hipStream_t s) {
    using A = typename Val<VT>::A;
    constexpr bool kWide = std::is_same<A, double>::value;
    constexpr int kRR2 = kWide ? 0 : 2, kRR4 = kWide ? 3 : 4;
    const int rr = d.row_reduce;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlockThreads), 0, s, d, a, b, (const A *)x, (A *)y);
    };
    auto by_rr = [&](auto agg) {
        constexpr int AG = decltype(agg)::value;
        if (rr == 2) go(spmv_quad_kernel<VT, AG, kRR2, LT, SC>);
        else if (rr == 3) go(spmv_quad_kernel<VT, AG, 3, LT, SC>);
        else if (rr == 4) go(spmv_quad_kernel<VT, AG, kRR4, LT, SC>);
        else go(spmv_quad_kernel<VT, AG, 0, LT, SC>);
    };
    if (d.col_agg == 3) by_rr(std::integral_constant<int, 3>());
    else if (d.col_agg == 2) by_rr(std::integral_constant<int, 2>());
    else if (d.col_agg) by_rr(std::integral_constant<int, 1>());
    else by_rr(std::integral_constant<int, 0>());
    return hipGetLastError();
}

template <int VT>
hipError_t spmv_vt(const DevView &d, double alpha, const void *x, double beta, void *y, hipStream_t s) {
    using A = typename Val<VT>::A;
    hipError_t e = prepass<A>(d, beta, y, 1, 1, s);
    if (e != hipSuccess) return e;
    if (d.nwaves <= 0) return hipSuccess;
    const int nb = (d.nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
    // row sums: FP32 LDS atomics are slow where many lanes of a pass hit one row (long runs),
    // the segmented scan costs the same whatever the runs; the handle holds the choice
    const A a = (A)alpha, b = (A)beta;
    if (d.scatter) {
        return spmv_quad_launch<VT, 4, true>(d, a, b, x, y, nb, s);
    } else if (d.natural_order && d.spmv_kernel == 2) {
        if (d.tile_lt == 3) return spmv_quad_launch<VT, 3>(d, a, b, x, y, nb, s);
        return spmv_quad_launch<VT, 4>(d, a, b, x, y, nb, s);
    } else if (d.natural_order && d.spmv_kernel == 1) {
        if (d.col_agg)
            hipLaunchKernelGGL((spmv_rows_kernel<VT, true>), dim3(nb), dim3(kBlockThreads), 0, s, d, a, b,
                               (const A *)x, (A *)y);
        else
            hipLaunchKernelGGL((spmv_rows_kernel<VT, false>), dim3(nb), dim3(kBlockThreads), 0, s, d, a, b,
                               (const A *)x, (A *)y);
    } else if (d.natural_order) {
        if (d.tile_lt == 3) return spmv_stream_launch<VT, 3>(d, a, b, x, y, nb, s);
        return spmv_stream_launch<VT, 4>(d, a, b, x, y, nb, s);
    } else
        hipLaunchKernelGGL(spmv_kernel<VT>, dim3(nb), dim3(kBlockThreads), 0, s, d, (A)alpha, (A)beta,
                           (const A *)x, (A *)y);
    return hipGetLastError();
}

// ---- k right-hand sides on the matrix cores (natural order) ----------------
//
// Y = alpha*A*X + beta*Y, KC columns of X per launch slice (blockIdx.y).  Every
// tile, whatever its storage format, is a 16 x 16 block of A; times the tile's
// 16 rows of X (a 16 x KC block) it is a small dense contraction, done on the
// matrix cores as four 16x16x4 MFMA steps per 16 output columns.  The panel's
// 16 x KC output block stays in the MFMA accumulators while the wavefront walks
// the panel's tiles and is written to Y when the panel changes.  COO and CSR
// tiles are expanded into a zero-filled 16 x 16 operand in LDS (their one-byte
// codes give row and column, Algorithm 3); Dense tiles are the operand already
// (Algorithm 4).  A tile whose staged X block holds an Inf or NaN is multiplied
// entry by entry instead, so a zero fill never meets it.
//
// Loads run NS - 1 tiles ahead: after tile t is multiplied, the entries and
// the X block of tile t+NS-1 and the column indices of tile t+NS are issued,
// so NS - 2 tiles are multiplied while they are in flight.  The loop is
// unrolled by NS so each tile's registers are fixed, and every load is issued
// on every path (addresses clamped into the range).

// operand and accumulator layouts (see Mfma): lane l holds A[l % 16][4kb + l / 16]
// and B[4kb + l / 16][l % 16] in step kb
// X32: every element of X lies within 4 GiB of X, so its address is X plus a 32-bit byte offset
// LT = 3 (8 x 8 tiles): the tile sits in the top-left corner of the 16 x 16 operand, only its
// columns' two 4-wide MFMA steps run and only the accumulator rows of its 8 panel rows are written.
template <int VT, int KC, bool AGG, int NS, bool X32, int LT>
__global__ __launch_bounds__(kBlockThreads) void spmm_mfma_kernel(DevView d, typename Val<VT>::A alpha,
                                                                  typename Val<VT>::A beta,
                                                                  const typename Val<VT>::A *__restrict__ X,
                                                                  int64_t ldx, typename Val<VT>::A *__restrict__ Y,
                                                                  int64_t ldy, int k) {
    using A = typename Val<VT>::A;
    using C = typename Mfma<A>::C;
    constexpr int VS = Val<VT>::kSize;
    constexpr int NB = KC / 16;  // 16-column output blocks
    constexpr int TS = 1 << LT;  // tile size
    constexpr int KB = TS / 4;   // 4-column MFMA steps per tile
    constexpr int MW = TS * TS / 32;  // bitmap words of a Dense tile
    using CI = typename std::conditional<LT == 4, u32x4, i32x2>::type;  // a lane's KB original columns
    static_assert(KC == 16 || KC == 32, "16 or 32 columns per slice");
    static_assert(LT == 3 || LT == 4, "16 x 16 or 8 x 8 tiles");
    __shared__ __align__(16) A dense_all[kWavesPerBlock][256];
    __shared__ A cs_all[kWavesPerBlock][16 * KC];
    __shared__ A xs_all[kWavesPerBlock][16 * KC];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int w = xcd_block(blockIdx.x, gridDim.x, d.xcd_chunk) * kWavesPerBlock + wid;
    if (w >= d.nwaves) return;
    const int t0 = d.wave_ptr[w], t1 = d.wave_ptr[w + 1];
    if (t0 >= t1) return;
    A *dense = dense_all[wid];
    A *cs = cs_all[wid];
    A *xs = xs_all[wid];
    const int j0 = blockIdx.y * KC;
    const int kc = min(KC, k - j0);
    const int lr = lane & 15, lg = lane >> 4;
    const int p_first = d.tile_row[t0], p_last = d.tile_row[t1 - 1];
    const bool sh_first = d.panel_shared[p_first] != 0, sh_last = d.panel_shared[p_last] != 0;

    // per-tile loads of one stage; the tile record arrives a stage before the entries need it.
    // Lane l takes entries 4l .. 4l+3 of a COO/CSR tile (codes as one dword) or elements 4l .. 4l+3
    // of a Dense tile (row l / 4, columns 4(l % 4) ..), so a stage is about a dozen wave loads and
    // four stages stay within the 63 vector loads a wavefront can have in flight.
    struct Stage {
        i32x4 rec;      // {vp low, vp high | type << 16 | (nnz - 1) << 18, panel, column block}
        CI ci;          // aggregation: original columns lg, lg + 4, ... of the tile
        A ev[4];        // values of entries (elements) 4l .. 4l+3
        uint32_t ec;    // COO/CSR: codes of entries 4l .. 4l+3; Dense: occupancy bitmap word l % MW
        A xb[NB][4];    // B operands: X[column 4kb + lg][j0 + 16ob + lr] (kb < KB)
    };
    auto issue_idx = [&](Stage &S, int t) __attribute__((always_inline)) {
        const int tc = min(t, t1 - 1);
        S.rec = reinterpret_cast<const i32x4 *>(d.tile_rec)[tc];
        if constexpr (AGG) S.ci = reinterpret_cast<const CI *>(d.tile_cols)[4 * (size_t)tc + lg];
    };
    auto rec_ty = [](int y) { return (y >> 16) & 3; };
    auto rec_nz = [](int y) { return ((y >> 18) & 0xFF) + 1; };
    auto issue_ent = [&](Stage &S) __attribute__((always_inline)) {
        const int y = __builtin_amdgcn_readfirstlane(S.rec.y);
        const int nz = rec_nz(y), ty = rec_ty(y);
        const int64_t vp = ((int64_t)(y & 0xFFFF) << 32) | (uint32_t)__builtin_amdgcn_readfirstlane(S.rec.x);
        const uint8_t *base = d.payload + vp;
        const int hb = ty == 1 ? TS : 0;
        const int e = 4 * lane < nz ? 4 * lane : 0;  // lanes past the tile re-read its first entries
        const uint8_t *vals = ty == 2 ? base : base + hb + nz + pad_bytes(hb + nz, VS);
        const int vi = ty == 2 ? (4 * lane < TS * TS ? 4 * lane : 0) : e;
        S.ec = ty == 2 ? reinterpret_cast<const uint32_t *>(base + TS * TS * VS)[lane & (MW - 1)]
                       : *reinterpret_cast<const uint32_t *>(base + hb + e);
        Val<VT>::load4(vals, vi, S.ev);
    };
    auto issue_x = [&](Stage &S) __attribute__((always_inline)) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            int col;
            if constexpr (AGG) {
                col = (int)S.ci[kb];
            } else {
                const int64_t c = ((int64_t)__builtin_amdgcn_readfirstlane(S.rec.w) << LT) + 4 * kb + lg;
                col = c < d.n ? (int)c : 0;
            }
            if constexpr (X32) {
                const uint32_t row = (uint32_t)col * (uint32_t)ldx;
#pragma unroll
                for (int ob = 0; ob < NB; ++ob) {
                    const uint32_t off = (row + (uint32_t)min(j0 + 16 * ob + lr, k - 1)) * (uint32_t)sizeof(A);
                    S.xb[ob][kb] = *reinterpret_cast<const A *>(reinterpret_cast<const char *>(X) + off);
                }
            } else {
                const A *xr = X + (int64_t)col * ldx;
#pragma unroll
                for (int ob = 0; ob < NB; ++ob) S.xb[ob][kb] = xr[min(j0 + 16 * ob + lr, k - 1)];
            }
        }
    };

    C acc[NB];
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) acc[ob] = C{A(0), A(0), A(0), A(0)};
    auto flush = [&](int p) {
        const bool shared = (p == p_first && sh_first) || (p == p_last && sh_last);
#pragma unroll
        for (int ob = 0; ob < NB; ++ob) {
            const int col = 16 * ob + lr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = ((int64_t)p << LT) + Mfma<A>::row(lane, v);
                if (Mfma<A>::row(lane, v) < TS && row < d.m && col < kc) {
                    A *yp = Y + row * ldy + j0 + col;
                    if (shared) {
                        global_add(yp, alpha * acc[ob][v]);
                    } else {
                        A out = alpha * acc[ob][v];
                        if (beta != A(0)) out += beta * *yp;
                        *yp = out;
                    }
                }
            }
            acc[ob] = C{A(0), A(0), A(0), A(0)};
        }
    };

    // entry-by-entry product of a tile whose X block is not finite: the accumulators and the X
    // block go through LDS and the entries come from the stage's registers by cross-lane reads, lanes
    // over the KC columns.  No global loads, so the counts of the loads in flight stay exact.
    auto exact_tile = [&](const Stage &S) __attribute__((always_inline)) {
        const int y = __builtin_amdgcn_readfirstlane(S.rec.y);
        const int nz = rec_nz(y), ty = rec_ty(y);
        const A v0 = S.ev[0], v1 = S.ev[1], v2 = S.ev[2], v3 = S.ev[3];
        const int ec = (int)S.ec;
#pragma unroll
        for (int ob = 0; ob < NB; ++ob) {
#pragma unroll
            for (int v = 0; v < 4; ++v) cs[Mfma<A>::row(lane, v) * KC + 16 * ob + lr] = acc[ob][v];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) xs[(4 * kb + lg) * KC + 16 * ob + lr] = S.xb[ob][kb];
        }
        __builtin_amdgcn_wave_barrier();
        // Dense: ec of lane i holds word i % MW of the occupancy bitmap and element e = TS r + c is
        // value e % 4 of lane e / 4; COO/CSR: entry e is byte e % 4 of ec and value e % 4 of lane e / 4
        const int n = ty == 2 ? TS * TS : nz;
        for (int e = 0; e < n; ++e) {
            int r, c, src, j;
            if (ty == 2) {
                if (!((__shfl(ec, e >> 5) >> (e & 31)) & 1)) continue;
                r = e >> LT;
                c = e & (TS - 1);
                src = e >> 2;
                j = e & 3;
            } else {
                const int code = (__shfl(ec, e >> 2) >> (8 * (e & 3))) & 0xFF;
                r = code & 15;
                c = code >> 4;
                src = e >> 2;
                j = e & 3;
            }
            const A sel = j == 0 ? v0 : j == 1 ? v1 : j == 2 ? v2 : v3;
            const A v = __shfl(sel, src);
            if (lane < KC) cs[r * KC + lane] += v * xs[c * KC + lane];
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[ob][v] = cs[Mfma<A>::row(lane, v) * KC + 16 * ob + lr];
        __builtin_amdgcn_wave_barrier();
    };

    int cur = -1;
    auto multiply = [&](const Stage &S) __attribute__((always_inline)) {
        const int p = __builtin_amdgcn_readfirstlane(S.rec.z);
        if (p != cur) {
            if (cur >= 0) flush(cur);
            cur = p;
        }
        bool finite = true;
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) finite = finite && __builtin_isfinite(S.xb[ob][kb]);
        if (__ballot(!finite) != 0) {
            exact_tile(S);
            return;
        }
        const int y = __builtin_amdgcn_readfirstlane(S.rec.y);
        const int nz = rec_nz(y), ty = rec_ty(y);
        // the 16 x 16 operand in LDS, element (r, c) at r*16 + (c%4)*4 + c/4, so lane l reads its four
        // values A[lr][4kb + lg] as one contiguous group; COO/CSR tiles (and 8 x 8 Dense tiles, which
        // fill its top-left corner) are zero-filled first
        if (ty != 2 || TS != 16) {
#pragma unroll
            for (int i = 0; i < 4; ++i) dense[4 * lane + i] = A(0);
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int r, c;
            if (ty == 2) {
                r = (4 * lane + i) >> LT;
                c = (4 * lane + i) & (TS - 1);
            } else {
                const int code = (S.ec >> (8 * i)) & 0xFF;
                r = code & 15;
                c = code >> 4;
            }
            if (ty == 2 ? 4 * lane + i < TS * TS : 4 * lane + i < nz) dense[r * 16 + (c & 3) * 4 + (c >> 2)] = S.ev[i];
        }
        __builtin_amdgcn_wave_barrier();
        A a[4];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) a[kb] = dense[lr * 16 + lg * 4 + kb];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) acc[ob] = Mfma<A>::step(a[kb], S.xb[ob][kb], acc[ob]);
    };

    // prologue: tiles t0 .. t0+NS-2 in flight, metadata and column indices of tile t0+NS-1
    Stage S[NS];
#pragma unroll
    for (int u = 0; u + 1 < NS; ++u) issue_idx(S[u], t0 + u);
#pragma unroll
    for (int u = 0; u + 1 < NS; ++u) {
        issue_ent(S[u]);
        issue_x(S[u]);
    }
    issue_idx(S[NS - 1], t0 + NS - 1);
    for (int t = t0; t < t1; t += NS) {
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const int tt = t + u;
            if (tt >= t1) break;
            multiply(S[u]);
            issue_idx(S[u], tt + NS);
            issue_ent(S[(u + NS - 1) % NS]);
            issue_x(S[(u + NS - 1) % NS]);
        }
    }
    if (cur >= 0) flush(cur);
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

template <int VT, int KC, bool AGG, int LT>
hipError_t spmm_mfma(const DevView &d, int k, double alpha, const void *X, int64_t ldx, double beta, void *Y,
                     int64_t ldy, hipStream_t s) {
    using A = typename Val<VT>::A;
    hipError_t e = prepass<A>(d, beta, Y, k, ldy, s);
    if (e != hipSuccess) return e;
    if (d.nwaves <= 0) return hipSuccess;
    const int nb = (d.nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
    const int ny = (k + KC - 1) / KC;
    constexpr bool kWide = std::is_same<A, double>::value;
    constexpr int NS = kWide && CB_TUNE_SPMM_STAGES > 2 ? CB_TUNE_SPMM_STAGES - 1 : CB_TUNE_SPMM_STAGES;  // FP64 stages are twice the registers
    const bool x32 = ((uint64_t)d.n * (uint64_t)ldx + (uint64_t)k) * sizeof(A) < ((uint64_t)1 << 32);
    if (x32)
        hipLaunchKernelGGL((spmm_mfma_kernel<VT, KC, AGG, NS, true, LT>), dim3(nb, ny), dim3(kBlockThreads), 0, s, d,
                           (A)alpha, (A)beta, (const A *)X, ldx, (A *)Y, ldy, k);
    else
        hipLaunchKernelGGL((spmm_mfma_kernel<VT, KC, AGG, NS, false, LT>), dim3(nb, ny), dim3(kBlockThreads), 0, s, d,
                           (A)alpha, (A)beta, (const A *)X, ldx, (A *)Y, ldy, k);
    return hipGetLastError();
}

template <int VT>
hipError_t spmm_vt(const DevView &d, int k, double alpha, const void *X, int64_t ldx, double beta, void *Y,
                   int64_t ldy, hipStream_t s) {
    if (d.natural_order && CB_TUNE_SPMM_MFMA) {
        const bool wide = k > 16 && CB_TUNE_SPMM_KC_MAX >= 32;
        if (d.tile_lt == 3) {
            if (d.col_agg)
                return wide ? spmm_mfma<VT, 32, true, 3>(d, k, alpha, X, ldx, beta, Y, ldy, s)
                            : spmm_mfma<VT, 16, true, 3>(d, k, alpha, X, ldx, beta, Y, ldy, s);
            return wide ? spmm_mfma<VT, 32, false, 3>(d, k, alpha, X, ldx, beta, Y, ldy, s)
                        : spmm_mfma<VT, 16, false, 3>(d, k, alpha, X, ldx, beta, Y, ldy, s);
        }
        if (d.col_agg)
            return wide ? spmm_mfma<VT, 32, true, 4>(d, k, alpha, X, ldx, beta, Y, ldy, s)
                        : spmm_mfma<VT, 16, true, 4>(d, k, alpha, X, ldx, beta, Y, ldy, s);
        return wide ? spmm_mfma<VT, 32, false, 4>(d, k, alpha, X, ldx, beta, Y, ldy, s)
                    : spmm_mfma<VT, 16, false, 4>(d, k, alpha, X, ldx, beta, Y, ldy, s);
    }
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
        case 3: return spmv_vt<3>(d, alpha, x, beta, y, stream);
        case 4: return spmv_vt<4>(d, alpha, x, beta, y, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spmm(const DevView &d, int vtype, int k, double alpha, const void *X, int64_t ldx, double beta,
                       void *Y, int64_t ldy, hipStream_t stream) {
    switch (vtype) {
        case 0: return spmm_vt<0>(d, k, alpha, X, ldx, beta, Y, ldy, stream);
        case 1: return spmm_vt<1>(d, k, alpha, X, ldx, beta, Y, ldy, stream);
        case 2: return spmm_vt<2>(d, k, alpha, X, ldx, beta, Y, ldy, stream);
        case 3: return spmm_vt<3>(d, k, alpha, X, ldx, beta, Y, ldy, stream);
        case 4: return spmm_vt<4>(d, k, alpha, X, ldx, beta, Y, ldy, stream);
        default: return hipErrorInvalidValue;
    }
}

namespace {
template <int VT, int AGG, int LT>
hipError_t batch_rr(const BatchJob *jobs, const int32_t *wave_job, int total, int rr, int quad, hipStream_t s) {
    constexpr bool kWide = std::is_same<typename Val<VT>::A, double>::value;
    const dim3 grid((unsigned)total), block(kBlockThreads);
    if (AGG == 3 && !quad) return hipErrorInvalidValue;  // per-batch column bases exist in quad batches only
    if (quad) {
        if (rr == 2)
            hipLaunchKernelGGL((spmv_qbatch_kernel<VT, AGG, kWide ? 0 : 2, LT>), grid, block, 0, s, jobs, wave_job,
                               total);
        else if (rr == 3)
            hipLaunchKernelGGL((spmv_qbatch_kernel<VT, AGG, 3, LT>), grid, block, 0, s, jobs, wave_job, total);
        else if (rr == 4)
            hipLaunchKernelGGL((spmv_qbatch_kernel<VT, AGG, kWide ? 3 : 4, LT>), grid, block, 0, s, jobs, wave_job,
                               total);
        else
            hipLaunchKernelGGL((spmv_qbatch_kernel<VT, AGG, 0, LT>), grid, block, 0, s, jobs, wave_job, total);
        return hipGetLastError();
    }
    constexpr int SAGG = AGG == 3 ? 2 : AGG;  // (not reached with AGG 3)
    if (rr == 1)
        hipLaunchKernelGGL((spmv_batch_kernel<VT, SAGG, 1, LT>), grid, block, 0, s, jobs, wave_job, total);
    else if (rr == 2)
        hipLaunchKernelGGL((spmv_batch_kernel<VT, SAGG, kWide ? 0 : 2, LT>), grid, block, 0, s, jobs, wave_job, total);
    else if (rr == 3)
        hipLaunchKernelGGL((spmv_batch_kernel<VT, SAGG, 3, LT>), grid, block, 0, s, jobs, wave_job, total);
    else if (rr == 4)
        hipLaunchKernelGGL((spmv_batch_kernel<VT, SAGG, kWide ? 3 : 4, LT>), grid, block, 0, s, jobs, wave_job, total);
    else
        hipLaunchKernelGGL((spmv_batch_kernel<VT, SAGG, 0, LT>), grid, block, 0, s, jobs, wave_job, total);
    return hipGetLastError();
}
template <int VT>
hipError_t batch_vt(const BatchJob *jobs, const int32_t *wave_job, int total, int agg, int rr, int quad, int lt,
                    hipStream_t s) {
    if (lt == 3)
        return agg == 3 ? batch_rr<VT, 3, 3>(jobs, wave_job, total, rr, quad, s)
               : agg == 2 ? batch_rr<VT, 2, 3>(jobs, wave_job, total, rr, quad, s)
               : agg      ? batch_rr<VT, 1, 3>(jobs, wave_job, total, rr, quad, s)
                          : batch_rr<VT, 0, 3>(jobs, wave_job, total, rr, quad, s);
    return agg == 3 ? batch_rr<VT, 3, 4>(jobs, wave_job, total, rr, quad, s)
           : agg == 2 ? batch_rr<VT, 2, 4>(jobs, wave_job, total, rr, quad, s)
           : agg      ? batch_rr<VT, 1, 4>(jobs, wave_job, total, rr, quad, s)
                      : batch_rr<VT, 0, 4>(jobs, wave_job, total, rr, quad, s);
}
}  // namespace

hipError_t launch_spmv_batch(const BatchJob *jobs, const int32_t *wave_job, int total, int vtype, int agg, int rr,
                             int quad, int lt, hipStream_t stream) {
    if (total <= 0) return hipSuccess;
    switch (vtype) {
        case 0: return batch_vt<0>(jobs, wave_job, total, agg, rr, quad, lt, stream);
        case 1: return batch_vt<1>(jobs, wave_job, total, agg, rr, quad, lt, stream);
        case 2: return batch_vt<2>(jobs, wave_job, total, agg, rr, quad, lt, stream);
        case 3: return batch_vt<3>(jobs, wave_job, total, agg, rr, quad, lt, stream);
        case 4: return batch_vt<4>(jobs, wave_job, total, agg, rr, quad, lt, stream);
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

hipError_t launch_read(const void *src, int64_t bytes, void *sink, hipStream_t stream) {
    const int64_t n16 = bytes / 16;
    const int64_t nw = (n16 + kReadSpan16 - 1) / kReadSpan16, nb = (nw + 256 / kWave - 1) / (256 / kWave);
    if (nb < 1) return hipSuccess;
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(read_kernel, dim3((unsigned)nb), dim3(256), 0, stream, (const uint4 *)src, n16, (uint4 *)sink);
    return hipGetLastError();
}

}  // namespace cbd
