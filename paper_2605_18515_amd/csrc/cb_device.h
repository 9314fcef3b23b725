// Device view of a converted matrix and the kernel launchers (internal to libcbspmv).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cbd {

// Pointers into the handle's single device allocation.  The tile arrays are in
// kernel order: wavefront w processes tiles [wave_ptr[w], wave_ptr[w+1]).
struct DevView {
    const int32_t *tile_row;      // panel (S = 1 << tile_lt rows) of the tile
    const int32_t *tile_col;      // column block (S columns), or aggregated chunk
    const int32_t *tile_nnz;
    const int64_t *tile_vp;       // byte offset of the tile's packed region
    const uint8_t *tile_type;     // 0 COO, 1 CSR, 2 Dense
    const int32_t *tile_xoff;     // col_agg only: restore_cols index of the tile's first column
    const uint8_t *payload;
    const int32_t *restore_cols;  // aggregated -> original column (col_agg only)
    const int32_t *cols_offset;   // npanels + 1 (col_agg only)
    const int32_t *wave_ptr;      // nwaves + 1
    const uint8_t *panel_shared;  // npanels
    const int32_t *prepass_list;  // nprepass
    const int32_t *batch_stream;  // natural order only: batch headers and tile records (cb_stream.h), 4 ints each
    const int32_t *batch_ptr;     // natural order only: first record of each work range, nwaves + 1
    const int32_t *tile_cols;     // natural order with col_agg: S original columns per tile
    const int32_t *tile_rec;      // natural order: {vp low, vp high | type << 16 | (nnz - 1) << 18, panel, column block}
    int64_t m, n;
    int32_t nwaves, npanels, nprepass;
    int32_t col_agg;              // 0 none; 1 aggregated, S 4-byte original columns per tile (tile_cols);
                                  // 2 aggregated, the streaming and quad kernels read tile_cbase +
                                  // tile_c16; 3 aggregated, the quad kernel reads tile_c16 + the batch
                                  // header's base (the other kernels read tile_cols, also present)
    int32_t natural_order;        // 1: kernel order = packing order, each work range one contiguous byte range
    int32_t row_reduce;           // streaming kernel row sums: 0 LDS atomics per entry, 1 DPP segmented scan,
                                  // 2 FP64 LDS atomics, 3 and 4 = 0 and 2 with two accumulator copies
    int32_t spmv_kernel;          // natural order: 0 the streaming kernel, 1 rows per lane, 2 the quad kernel
                                  // (batch_stream then holds quad batches)
    const int32_t *panel_tile;    // natural order: first tile of each panel, npanels + 1
    const int32_t *tile_cbase;    // col_agg 2: first original column of each tile
    const uint16_t *tile_c16;     // col_agg 2 and 3: S column offsets per tile from its base (2) or its
                                  // batch's (3), natural column order
    int32_t tile_lt;              // log2 of the tile size S: 4 (16 x 16 tiles) or 3 (8 x 8)
    int32_t scatter;              // Algorithm 2's groups streamed (CB_LB_PAPER_STREAM): quad batches in
                                  // scatter form, every tile's rows added into y with atomics
    int32_t xcd_chunk;            // workgroup-to-range mapping: 0 each XCD a contiguous eighth; c runs of c
    int32_t pad1;
    int64_t payload_alloc;        // readable bytes from payload (the structure's bytes and the padding after them)
    int64_t stream_alloc;         // readable bytes from batch_stream
};

// One product of a batched launch: y = alpha A x + beta y for the natural-order structure d, its
// work ranges at global workgroups wave_base .. wave_base + d.nwaves - 1 of the launch.
struct BatchJob {
    DevView d;
    const void *x;
    void *y;
    double alpha, beta;
    int32_t wave_base;
    int32_t pad;
};

// Products of several natural-order structures in one launch.  wave_job[b] (total entries, device
// memory) is the job of workgroup b; every job has kernel value code vtype, aggregation agg,
// row-sum mode rr, batch format (quad: 1 for spmv_kernel 2 structures, else 0) and tile size
// 1 << lt; y rows of shared panels must be prepared as for one product.
hipError_t launch_spmv_batch(const BatchJob *jobs, const int32_t *wave_job, int total, int vtype, int agg, int rr,
                             int quad, int lt, hipStream_t stream);

// vtype: 0 = FP64 values, x, y double; 1 = FP32 values; 2 = BF16 values (x, y float);
// 3 = FP32 values, 4 = BF16 values with x, y double and FP64 arithmetic
hipError_t launch_spmv(const DevView &d, int vtype, double alpha, const void *x, double beta, void *y,
                       hipStream_t stream);
hipError_t launch_spmm(const DevView &d, int vtype, int k, double alpha, const void *X, int64_t ldx, double beta,
                       void *Y, int64_t ldy, hipStream_t stream);
hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t stream);
hipError_t launch_read(const void *src, int64_t bytes, void *sink, hipStream_t stream);

}  // namespace cbd
