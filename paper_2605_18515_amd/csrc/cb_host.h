// Host-side CB structure and converter interface (internal to libcbspmv).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "cb_stream.h"
#include "cbspmv.h"

namespace cbh {

constexpr int kBlk = 16;          // Section 3.1: 16 x 16 sub-blocks (the default; 8 x 8 on request)
constexpr int kSuperSparse = 32;  // Section 3.3.1: fewer than 32 non-zeros (on the 16 x 16 partition)
constexpr int kTileAlign = 16;    // every tile region starts on a 16-byte boundary
// occupancy bitmap of a Dense S x S tile: one bit per element
constexpr int dense_mask_bytes(int blk) { return blk * blk / 8; }
constexpr int kTileCost = 8;      // per-tile overhead, in non-zero equivalents, for range balancing
constexpr int64_t kQuadMaxCols = (int64_t(1) << 29) - 16;  // the quad kernel reads x at 32-bit byte offsets

// load-balance modes whose wavefront ranges are contiguous byte ranges of the payload, cut into
// batches (all but Algorithm 2's tile-at-a-time form), and those whose kernel order is the natural
// (panel, column) order
inline bool streamed_lb(int lb) { return lb != CB_LB_PAPER; }
inline bool natural_lb(int lb) { return lb == CB_LB_NONE || lb == CB_LB_CONTIGUOUS; }

struct HostStructure {
    int64_t m = 0, n = 0, nnz = 0;
    int vtype = CB_VALUE_F64;
    int vsize = 8;
    int col_agg = 0;
    double share = 0.0;
    int64_t plain_tiles = 0;
    int lb_mode = CB_LB_CONTIGUOUS;
    int quantum_tiles = 8;
    int blk = kBlk;  // tile size S: panels of S rows, S x S tiles (16 or 8)
    int lt = 4;      // log2(S)
    int64_t npanels = 0, ntiles = 0;
    // kernel order (after load balance)
    std::vector<int32_t> tile_row, tile_col, tile_nnz, tile_ori;
    std::vector<int32_t> tile_xoff;  // aggregation only: cols_offset[row] + S * col (restore_cols index of the tile)
    std::vector<int64_t> tile_vp;
    std::vector<uint8_t> tile_type;
    std::vector<uint8_t> payload;
    std::vector<int32_t> restore_cols, cols_offset;
    std::vector<int32_t> quantum_ptr, wave_ptr;
    std::vector<uint8_t> panel_shared;
    std::vector<int32_t> prepass_list;
    // batch records of the streaming kernel (natural-order modes only): 4 ints per record,
    // batch_ptr[w] = first record of work range w
    std::vector<int32_t> batch_stream, batch_ptr;
    // column aggregation with the streaming kernel: S original columns per tile, kernel order
    std::vector<int32_t> tile_cols;
    // cols16: every tile's first original column, and its S columns as offsets from it (natural
    // column order; columns past the tile's last: 0), read by the SpMV kernels instead of tile_cols
    int cols16 = 0;
    std::vector<int32_t> tile_cbase;
    std::vector<uint16_t> tile_c16;
    // natural-order modes: one 16-byte record per tile for the k-right-hand-side kernel
    // {vp low word, vp high 16 bits | type << 16 | (nnz - 1) << 18, panel, column block}
    std::vector<int32_t> tile_rec;
    // counts kept when the big arrays move to the device
    int64_t payload_bytes = 0, nrestore = 0, nquanta = 0, nwaves = 0, nprepass = 0, nshared = 0;
    int64_t nbatches = 0, nrecords = 0;
    int64_t tiles_fmt[3] = {0, 0, 0};
    int64_t quantum_nnz_max = 0, wave_nnz_max = 0;
    double quantum_nnz_mean = 0, quantum_nnz_std = 0, wave_nnz_mean = 0, wave_nnz_std = 0;
    double convert_seconds = 0.0;
    int64_t flat_entries = 0, flat_runs = 0;  // COO/CSR entries and their (tile, row) runs
    int row_reduce = 0;                       // resolved: 0 LDS atomics, 1 DPP segmented scan, 2 FP64 atomics,
                                              // 3 and 4 = 0 and 2 with two accumulator copies
    int vector_f64 = 1;                       // x and y are double
    int xcd_chunk = 0;                        // resolved workgroup-to-range mapping (0 eighths, c runs of c)
    int spmv_kernel = 0;                      // resolved: 0 entries per lane, 1 rows per lane
    // natural order: first tile of every panel (npanels + 1)
    std::vector<int32_t> panel_tile;
};

int padding(int64_t index_bytes, int vsize);
int64_t region_bytes(int fmt, int64_t nnz, int vsize, int blk);
uint32_t f32_bits_rne(double v);
uint16_t bf16_bits_rne(double v);

// Bytes of payload one work range of the streaming kernel may span: its batch records and the
// kernel address the range with 32-bit offsets (plus the readable padding past the payload's end).
constexpr int64_t kMaxRangeSpan = ((int64_t)1 << 31) - 2 * cbs::kPayloadPad;

// max_range_span: the limit above (a smaller one only in the converter's own tests).
cb_status_t convert(int64_t m, int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                    const double *values, const cb_options_t &opt, HostStructure &out, std::string &err,
                    int64_t max_range_span = kMaxRangeSpan);
cb_status_t export_csr(const HostStructure &s, int64_t *row_ptr, int32_t *col_idx, void *values, std::string &err);
void fill_info(const HostStructure &s, cb_info_t &info);
int64_t spmv_bytes(const HostStructure &s);
// message returned by cb_last_error on this thread (set by the parts of the library outside capi.cpp)
void set_last_error(const std::string &msg);

}  // namespace cbh
