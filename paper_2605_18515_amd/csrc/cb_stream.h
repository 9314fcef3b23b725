// Batch records of the streaming SpMV kernel, shared by the converter (which
// writes them) and the kernel (which reads them).  Internal to libcbspmv.
//
// With the contiguous or no load balance the kernel order is the packing
// order, so a wavefront's tiles occupy one contiguous byte range of the
// payload.  The converter cuts every wavefront range into batches and writes,
// per batch, one 16-byte header followed by one 16-byte record per tile:
//
//   header  {re, pb, nt | nflat << 8 | ndense << 16 | done << 24, etot}
//     re     end of the batch's payload bytes, relative to the range's first
//            payload byte (the batch starts where the previous one ended)
//     pb     first panel of the batch
//     nt     tiles; nflat of them COO or CSR, ndense Dense
//     done   bit k: panel pb + k has its last tile of this range in the batch
//     etot   COO and CSR entries of the batch (the flat entry stream)
//   flat record (COO and CSR tiles, in order)  {pk, end, 0, xo}
//     the tile's entries are flat entries es .. end of the batch, and flat
//     entry E has its one-byte code at payload byte cpos + E and its value at
//     byte vpos + size(Val) * E (relative to the range's first payload byte);
//   dense record (Dense tiles, after the flat ones)  {pk, 0, rel, xo}
//     rel    the tile's first payload byte (relative)
//   pk       (cpos mod 4096) | (vpos mod 4096) << 12 | slot << 24 | ti << 27
//            (0 positions for Dense tiles): the kernel addresses its 4 KB
//            payload ring modulo 4096, so one 32-bit word per entry pass
//   slot     panel & (kBatchPanels - 1): the panel's accumulator in the kernel
//   ti       the tile's position in the batch (tiles in kernel order), which is
//            where its 16 x values land in the kernel's x area
//   xo       restore_cols index of the tile's first column under column
//            aggregation (cols_offset[panel] + 16 * chunk), else its column block
//
// With column aggregation the converter also writes tile_cols: for every tile in
// kernel order its 16 original columns (restore_cols[xo .. xo + 15], the columns
// past a panel's last one replaced by that panel's first), local column c at
// position (c mod 4) * 4 + c / 4 of the tile's 16, so the x column indices of a
// batch are one contiguous 64-byte-per-tile block and the four columns q, q + 4,
// q + 8, q + 12 of one matrix-core operand lane are adjacent.
#pragma once

#ifndef CB_TUNE_BATCH_TILES
#define CB_TUNE_BATCH_TILES 16
#endif
#ifndef CB_TUNE_RING_CHUNKS
#define CB_TUNE_RING_CHUNKS 4
#endif

namespace cbs {

constexpr int kChunk = 1024;      // payload bytes one wavefront-wide 16-byte load covers
constexpr int kRingChunks = CB_TUNE_RING_CHUNKS;  // payload chunks a batch may touch (the kernel's LDS ring)
constexpr int kRingBits = kRingChunks == 2 ? 11 : kRingChunks == 4 ? 12 : 13;  // log2 of the ring's bytes: the
                                                                              // width of the packed positions
static_assert(kChunk * kRingChunks == 1 << kRingBits, "packed positions address the ring");
constexpr int kBatchTiles = CB_TUNE_BATCH_TILES;  // tiles per batch (at most 16: 4-bit positions in the record word)
static_assert(kBatchTiles >= 4 && kBatchTiles <= 16 && kBatchTiles % 4 == 0, "tile positions take 4 bits");
constexpr int kBatchPanels = 4;   // consecutive panels a batch may touch (accumulator slots)
constexpr int kRecordPad = kBatchTiles + 1;  // records readable past the end of the stream
constexpr int kPayloadPad = 2048;            // payload and restore_cols bytes readable past their ends

// ---- quad stream (the quad kernel, spmv_kernel = 2) --------------------------
//
// The same work ranges cut into batches of at most kQTiles tiles, kBatchPanels consecutive panels
// and kQPasses * 64 quads.  A quad is four consecutive entries of one tile: a COO or CSR tile of nz
// entries holds ceil(nz / 4) quads (its last one partly empty), a Dense tile 64 (entries e = 4q ..
// 4q + 3 of its row-major 256, occupancy bits honoured).  The quads of a batch are numbered Q = 0 ..
// qtot - 1 in tile order; in pass p of the kernel lane l takes quad 64 p + l.
//
//   header  {pb, nt | np << 8 | done << 16, qtot, cbase}
//     pb     first panel of the batch; nt tiles; np = ceil(qtot / 64) passes
//     done   bit k: panel pb + k has its last tile of this range in the batch
//     cbase  with per-batch 2-byte column offsets (cols16 2): the batch's lowest original column,
//            which its tiles' offsets are taken from; else 0
//   record of tile i of the batch (i = 0 .. nt - 1, kernel order)  {cb, vb, lim, meta}
//     meta   slot | qs << 2 | dense << 15, with slot = panel & (kBatchPanels - 1) and qs the
//            tile's first quad
//     COO / CSR:  the four codes of quad Q are the dword at payload byte cb + 4 Q, its four values
//                 start at vb + 4 * size(Val) * Q (bytes relative to the range's first payload
//                 byte), and entry 4 Q + j exists iff 4 Q + j < lim (= 4 qs + nz)
//     Dense:      cb = the tile's occupancy bitmap, vb as above; the four bits of quad Q are
//                 nibble Q - qs of the bitmap
// The x area of the kernel holds the batch's tiles' 16 x values each, tile i at 16 i.
//
// Scatter form (Algorithm 2's groups streamed, CB_LB_PAPER_STREAM): the tiles of a batch may come
// from any panels; the batch limits are kQTiles tiles and kQPasses * 64 quads.
//   header  {0, nt | np << 8, qtot, cbase}
//   record  {cb, vb, panel, i | qs << 5 | dense << 15 | lim << 16}
//     i      the tile's position in the batch: its accumulator slot and x-area place
//     panel  the tile's panel, whose rows the tile's sums are added into after the batch
//     cb, vb, qs, dense, lim as above (lim = 4 qs + nz < 2^13)
#ifndef CB_TUNE_QTILES
#define CB_TUNE_QTILES 16
#endif
#ifndef CB_TUNE_QPASSES
#define CB_TUNE_QPASSES 3
#endif
constexpr int kQTiles = CB_TUNE_QTILES;    // tiles per quad batch (x-area slots)
constexpr int kQPasses = CB_TUNE_QPASSES;  // passes of 64 quads per batch (the kernel's payload registers)
static_assert(kQTiles % 4 == 0 && kQTiles <= 32, "x gathers take four tiles; tile positions fit the x-area index");
constexpr int kQRecordPad = kQTiles + 1;  // records readable past the end of the quad stream
static_assert(kQPasses * 64 <= 1023, "first quads take 10 bits of the record word");
static_assert(kQPasses >= 1 && kQPasses <= 4, "the quad kernel's tile-start marks take one byte per pass of a 32-bit word");
constexpr int kStreamRecordPad = kQRecordPad > kRecordPad ? kQRecordPad : kRecordPad;  // both batch formats

}  // namespace cbs
