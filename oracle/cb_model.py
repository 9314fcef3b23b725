"""Conversion oracle for the CB structure -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the benchmark's CPU baseline
may import this module.  It shares no code with the GPU library and imports
nothing from it.  It restates, step by step and in the paper's order and
notation, how CB-SpMV turns a sparse matrix into its two-level tile structure
(Section 3, Fig. 7):

  1. uniform 16 x 16 partition into sub-blocks ("tiles") keyed like a block
     COO (Section 3.1; 8 x 8 as the other sub-block size the library offers);
  2. the th0 decision on the share of super-sparse tiles and, when taken,
     block-aware column aggregation per panel of tile rows (Section 3.3.1);
  3. per-tile format selection with th1 / th2 (Section 3.3.2);
  4. intra-block data aggregation: packed 4+4-bit coordinates, padding and
     values behind a virtual pointer (Section 3.2, Algorithm 3 unpacking);
  5. inter-thread-block load balance with a priority queue (Section 3.4,
     Algorithm 2).

Where the paper is silent the module takes the readings listed in the design
notes (marked "reading:" below).  Plain Python loops over tiles keep it easy to
check by eye; it is meant for matrices of a few thousand tiles.
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass, field

import numpy as np

BLK = 16              # Section 3.1: uniform 16 x 16 sub-blocks
BLK_SIZES = (8, 16)   # sub-block sizes the library offers (8: the same one-byte codes, fewer slots)
SUPER_SPARSE = 32     # Section 3.3.1: "super-sparse" = fewer than 32 non-zeros
TH0 = 0.15            # Section 3.3.1
TH1 = 32              # Section 3.3.2: COO below th1
TH2 = 128             # Section 3.3.2: Dense above th2
WARPS_PER_TB = 8      # Section 3.4, Algorithm 2: eight sub-blocks per thread block

COO, CSR, DENSE = 0, 1, 2
VALUE_SIZE = {"f64": 8, "f32": 4, "bf16": 2}
TILE_ALIGN = 16       # reading: every tile region starts on a 16-byte boundary


@dataclass
class Tile:
    panel: int                 # blk_row_idx: index of the panel (blk rows)
    tcol: int                  # blk_col_idx: column-block (or aggregated chunk) index
    entries: list              # [(local_row, local_col, entry_index_in_input)], row-major
    fmt: int = COO

    @property
    def nnz(self) -> int:
        return len(self.entries)


@dataclass
class Model:
    m: int
    n: int
    col_agg: bool
    share: float                       # super-sparse share on the plain 16 x 16 partition
    tiles: list                        # natural order: (panel, tcol) ascending
    restore_cols: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    cols_offset: np.ndarray = field(default_factory=lambda: np.zeros(1, np.int64))
    blk: int = BLK                     # sub-block size: panels of blk rows, tiles blk x blk


# ---- Section 3.1: uniform 16 x 16 partition -------------------------------

def csr_rows(row_ptr: np.ndarray) -> np.ndarray:
    m = row_ptr.shape[0] - 1
    return np.repeat(np.arange(m, dtype=np.int64), np.diff(row_ptr))


def plain_tiles(row_ptr, col_idx, blk: int = BLK) -> dict:
    """Sub-block of entry (r, c) is (r // blk, c // blk); its local coordinates are
    (r % blk, c % blk).  Returns {(panel, cb): [(lr, lc, t), ...]} with entries in
    row-major order inside each tile."""
    rows = csr_rows(row_ptr)
    tiles: dict = {}
    for t in range(col_idx.shape[0]):
        r, c = int(rows[t]), int(col_idx[t])
        tiles.setdefault((r // blk, c // blk), []).append((r % blk, c % blk, t))
    for ent in tiles.values():
        ent.sort()
    return tiles


# ---- Section 3.3.1: th0 decision and block-aware column aggregation --------

def super_sparse_share(tiles: dict) -> float:
    """Share of non-empty sub-blocks with fewer than 32 non-zeros (reading: always
    taken on the paper's 16 x 16 partition, whatever sub-block size the structure
    then uses -- the paper defines super-sparse for 16 x 16 sub-blocks only)."""
    if not tiles:
        return 0.0
    return sum(1 for e in tiles.values() if len(e) < SUPER_SPARSE) / len(tiles)


def decide_col_agg(share: float, th0: float = TH0, mode: int = -1) -> bool:
    """mode -1: the paper's rule -- aggregation is skipped when the share of
    super-sparse sub-blocks is low, i.e. below th0 (reading: applied iff
    share >= th0, decided once for the whole matrix).  mode 0/1 force it."""
    if mode == 0:
        return False
    if mode == 1:
        return True
    return share >= th0


def aggregate_columns(m: int, row_ptr, col_idx, blk: int = BLK):
    """Per panel of blk rows, drop the columns that hold no entry and shift the
    rest left (Fig. 5(b)); restore_cols maps an aggregated column back to the
    original one and cols_offset marks where each panel's list starts.

    reading: the aggregated columns of panel p are its distinct original columns
    in ascending order; aggregated column a lands in chunk a // blk at local
    column a % blk, and the original column is
    restore_cols[cols_offset[p] + blk * chunk + local_col]."""
    npanels = (m + blk - 1) // blk
    rows = csr_rows(row_ptr)
    restore, offsets = [], [0]
    tiles: dict = {}
    for p in range(npanels):
        lo, hi = int(row_ptr[p * blk]), int(row_ptr[min(m, (p + 1) * blk)])
        cols_p = sorted(set(int(c) for c in col_idx[lo:hi]))
        rank = {c: a for a, c in enumerate(cols_p)}
        restore.extend(cols_p)
        offsets.append(offsets[-1] + len(cols_p))
        for t in range(lo, hi):
            a = rank[int(col_idx[t])]
            tiles.setdefault((p, a // blk), []).append((int(rows[t]) % blk, a % blk, t))
    for ent in tiles.values():
        ent.sort()
    return np.array(restore, dtype=np.int32), np.array(offsets, dtype=np.int64), tiles


# ---- Section 3.3.2: format selection --------------------------------------

def select_format(nnz: int, th1: int = TH1, th2: int = TH2) -> int:
    """COO when nnz < th1, Dense when nnz > th2, CSR otherwise."""
    if nnz < th1:
        return COO
    if nnz > th2:
        return DENSE
    return CSR


def build(m: int, n: int, row_ptr, col_idx, col_agg_mode: int = -1, th0: float = TH0,
          th1: int = TH1, th2: int = TH2, blk: int = BLK) -> Model:
    """Steps 1-3 of the pipeline in the paper's order (Fig. 7): partition,
    aggregation decision and aggregation, format per sub-block.  blk is the
    sub-block size (16 in the paper, 8 the library's other choice)."""
    if blk not in BLK_SIZES:
        raise ValueError("sub-block size must be one of %s" % (BLK_SIZES,))
    row_ptr = np.asarray(row_ptr)
    col_idx = np.asarray(col_idx)
    share = super_sparse_share(plain_tiles(row_ptr, col_idx, BLK))
    agg = decide_col_agg(share, th0, col_agg_mode)
    if agg:
        restore, offsets, tiles = aggregate_columns(m, row_ptr, col_idx, blk)
    else:
        restore, offsets, tiles = np.zeros(0, np.int32), np.zeros(1, np.int64), plain_tiles(row_ptr, col_idx, blk)
    order = sorted(tiles)
    out = [Tile(p, c, tiles[(p, c)], select_format(len(tiles[(p, c)]), th1, th2)) for (p, c) in order]
    return Model(m, n, agg, share, out, restore, offsets, blk)


# ---- Section 3.2 / Algorithm 3: intra-block data aggregation --------------

def padding(nnz_index_bytes: int, size_val: int) -> int:
    """Algorithm 3's padding: (nnz * size(Idx)) mod size(Val), replaced by
    size(Val) - that remainder when it is non-zero."""
    pad = nnz_index_bytes % size_val
    return size_val - pad if pad else 0


def pack_code(lr: int, lc: int) -> int:
    """4-bit row and 4-bit column in one byte; Algorithm 3 unpacks the row as
    the low nibble (b & 15) and the column as the high nibble (b >> 4)."""
    return (lc << 4) | lr


def unpack_code(b: int) -> tuple[int, int]:
    return b & 15, b >> 4


def tile_region_bytes(fmt: int, nnz: int, vtype: str, blk: int = BLK) -> int:
    """Bytes of one tile's packed region (before rounding to TILE_ALIGN).

    COO:   nnz codes, padding, nnz values.
    CSR:   blk one-byte row starts, nnz codes, padding, nnz values
           (reading: the paper gives no in-tile CSR layout).
    Dense: blk * blk values in row-major order, then a blk * blk / 8-byte
           occupancy bitmap so explicitly stored zeros survive (reading)."""
    sv = VALUE_SIZE[vtype]
    if fmt == COO:
        return nnz + padding(nnz, sv) + nnz * sv
    if fmt == CSR:
        return blk + nnz + padding(blk + nnz, sv) + nnz * sv
    return blk * blk * sv + blk * blk // 8


def layout(model: Model, vtype: str) -> tuple[list, int]:
    """Virtual pointers of the tiles in natural order: each region starts at
    the next 16-byte boundary after the previous one.  Returns (vps, total)."""
    vps, off = [], 0
    for t in model.tiles:
        vps.append(off)
        size = tile_region_bytes(t.fmt, t.nnz, vtype, model.blk)
        off += (size + TILE_ALIGN - 1) // TILE_ALIGN * TILE_ALIGN
    return vps, off


def value_bits(values: np.ndarray, vtype: str, rounder=None) -> np.ndarray:
    """Stored value bit patterns: FP64 as is; FP32 / BF16 through ``rounder``
    (the C oracle's round-to-nearest-even)."""
    if vtype == "f64":
        return np.ascontiguousarray(values, dtype=np.float64).view(np.uint64)
    if rounder is None:
        raise ValueError("a rounding function is needed for " + vtype)
    return rounder(values)


def pack(model: Model, values: np.ndarray, vtype: str, rounder=None) -> bytes:
    """Intra-block data aggregation (Section 3.2): every tile's codes, padding
    and values side by side in one byte buffer at its virtual pointer."""
    import struct

    sv = VALUE_SIZE[vtype]
    fmtc = {8: "<Q", 4: "<I", 2: "<H"}[sv]
    bits = value_bits(values, vtype, rounder)
    vps, total = layout(model, vtype)
    buf = bytearray(total)
    blk = model.blk
    for t, vp in zip(model.tiles, vps):
        if t.fmt == DENSE:
            mask = bytearray(blk * blk // 8)
            for lr, lc, idx in t.entries:
                e = lr * blk + lc
                struct.pack_into(fmtc, buf, vp + e * sv, int(bits[idx]))
                mask[e >> 3] |= 1 << (e & 7)
            buf[vp + blk * blk * sv: vp + blk * blk * sv + len(mask)] = mask
            continue
        codes = vp
        hdr = 0
        if t.fmt == CSR:
            hdr = blk
            for r in range(blk):
                buf[vp + r] = sum(1 for e in t.entries if e[0] < r)
            codes = vp + blk
        base_v = codes + t.nnz + padding(hdr + t.nnz, sv)
        for i, (lr, lc, idx) in enumerate(t.entries):
            buf[codes + i] = pack_code(lr, lc)
            struct.pack_into(fmtc, buf, base_v + i * sv, int(bits[idx]))
    return bytes(buf)


def decode_tile(buf: bytes, vp: int, fmt: int, nnz: int, vtype: str, blk: int = BLK) -> list:
    """Unpack one tile starting at virtual pointer vp: returns
    [(local_row, local_col, value_bits)] in storage order (Algorithm 3 for COO;
    row starts + codes for CSR; the occupancy bitmap for Dense)."""
    sv = VALUE_SIZE[vtype]
    fmtc = {8: "<Q", 4: "<I", 2: "<H"}[sv]
    import struct

    def val(off):
        return struct.unpack_from(fmtc, buf, off)[0]

    out = []
    if fmt == COO:
        base_v = vp + nnz + padding(nnz, sv)
        for i in range(nnz):
            lr, lc = unpack_code(buf[vp + i])
            out.append((lr, lc, val(base_v + i * sv)))
    elif fmt == CSR:
        starts = list(buf[vp:vp + blk]) + [nnz]
        codes = vp + blk
        base_v = codes + nnz + padding(blk + nnz, sv)
        for r in range(blk):
            for i in range(starts[r], starts[r + 1]):
                lr, lc = unpack_code(buf[codes + i])
                if lr != r:
                    raise ValueError("CSR tile: code row does not match row start")
                out.append((lr, lc, val(base_v + i * sv)))
    else:
        mask = buf[vp + blk * blk * sv: vp + blk * blk * sv + blk * blk // 8]
        for e in range(blk * blk):
            if (mask[e >> 3] >> (e & 7)) & 1:
                out.append((e // blk, e % blk, val(vp + e * sv)))
    return out


# ---- Section 3.4 / Algorithm 2: inter-thread-block load balance ------------

def lb_paper(nnz_per_blk, W: int = WARPS_PER_TB):
    """Algorithm 2.  Sort the sub-blocks by nnz, then hand them one by one to the
    thread block at the top of a min-heap keyed on its load; a thread block
    leaves the heap once it holds W sub-blocks.  Returns (end, order, T):
    end[i] = tb_id * W + warps for sub-block i (natural order), order = the
    sub-blocks sorted by end, T = number of thread blocks.

    readings: the sort is by descending nnz (largest first), stable on the
    original index; heap ties go to the lower tb_id; T = ceil(blocks / W); the
    heap loop is sequential."""
    nnz = list(nnz_per_blk)
    nb = len(nnz)
    T = (nb + W - 1) // W
    blk_idx = sorted(range(nb), key=lambda i: (-nnz[i], i))
    pq = [(0, tb, 0) for tb in range(T)]
    heapq.heapify(pq)
    end = [0] * nb
    for i in blk_idx:
        loads, tb_id, warps = heapq.heappop(pq)
        end[i] = tb_id * W + warps
        loads += nnz[i]
        warps += 1
        if warps < W:
            heapq.heappush(pq, (loads, tb_id, warps))
    order = sorted(range(nb), key=lambda i: end[i])
    return end, order, T


def lb_quantum_loads(nnz_per_blk, end, T: int, W: int = WARPS_PER_TB) -> np.ndarray:
    loads = np.zeros(T, dtype=np.int64)
    for i, e in enumerate(end):
        loads[e // W] += nnz_per_blk[i]
    return loads


# ---- Section 4.4.1: storage model ----------------------------------------

def bytes_model_cb(nnzb: int, nnz: int) -> int:
    """CB storage with every sub-block in COO: nnzb*(4+4+4+1+8) + nnz*(1+8)."""
    return nnzb * (4 + 4 + 4 + 1 + 8) + nnz * (1 + 8)


def bytes_model_csr(m: int, nnz: int) -> int:
    return (m + 1) * 4 + nnz * 4 + nnz * 8


def bytes_model_bsr(nnzb: int, blk_m: int) -> int:
    return 256 * 8 * nnzb + (blk_m + 1) * 4 + nnzb * 4
