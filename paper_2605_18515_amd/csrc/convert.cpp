// Host converter: CSR -> CB structure (Section 3, Fig. 7 order), CB -> CSR
// export and structure statistics.  Plain C++17, no HIP.
#include <sched.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <mutex>
#include <numeric>
#include <queue>
#include <thread>

#include "cb_host.h"

// Automatic work per wavefront range (non-zero equivalents): enough ranges to occupy every
// wavefront slot of the device about once (256 CUs x 22 resident wavefronts = 5632; aiming at 5120
// keeps a count that rounds up from spilling into a second, nearly empty round), no range below 256
// (a range's fixed cost, its pipeline fill, dominates shorter ones) and none above about 18 KB of
// codes and values (2048 entries of FP64 values, 3686 of FP32, 4096 of BF16): on the largest matrices
// shorter ranges balance the last round better, FP64 1.7-3.8 % faster than at 4096, while the
// smaller FP32/BF16 entries keep the longer ranges they measured best with.  Measured
// against 16384 ranges of at least 64: a 7-point operator on 100^3 nodes 27.6 against 34.2 us, on
// 50^3 6.5 against 11.4 us, a 64 x 64 Laplacian 3.3 against 2.9 us (graph replay), and the serving
// loop's batched products 1.38x the solves per second.
#ifndef CB_TUNE_MIN_WAVE_NNZ
#define CB_TUNE_MIN_WAVE_NNZ 256
#endif
#ifndef CB_TUNE_WAVE_RANGES
#define CB_TUNE_WAVE_RANGES 5120
#endif
// Matrices whose automatic ranges reach the cap run several rounds of wavefronts; there (unless each
// XCD takes an eighth of the ranges) the ranges
// of the last stretch shrink (guided self-scheduling: the remaining work / 2560, down to a quarter
// of the cap), so the last wavefronts to start end soon after the others instead of a whole range
// later.  Measured on the 3D block matrix: SpMM k = 8 and 32 7-8 % faster (FP32 and BF16 values),
// FP32 SpMV 1.4 %, the 192^3 Poisson operator 1.2 %, the FP64 block SpMV unchanged; remaining / 5120
// or / 10240 and floors of a half or an eighth of the cap measured between that and 1.6 % slower
// FP64 products (more, shorter ranges).
#ifndef CB_TUNE_TAPER_DIV
#define CB_TUNE_TAPER_DIV 2560
#endif
#ifndef CB_TUNE_TAPER_FLOOR
#define CB_TUNE_TAPER_FLOOR 4
#endif
#ifndef CB_TUNE_MAX_RANGE_BYTES
#define CB_TUNE_MAX_RANGE_BYTES 18432
#endif

namespace cbh {

namespace {

int default_threads() {
    cpu_set_t set;
    if (sched_getaffinity(0, sizeof(set), &set) == 0) {
        int c = CPU_COUNT(&set);
        if (c > 0) return c;
    }
    unsigned h = std::thread::hardware_concurrency();
    return h ? (int)h : 1;
}

// Runs fn(begin, end) over [0, n) in chunks of `grain`, handed out dynamically.
template <class F>
bool parallel_dynamic(int nthreads, int64_t n, int64_t grain, F &&fn, std::string &err) {
    if (n <= 0) return true;
    std::atomic<int64_t> next{0};
    std::atomic<bool> failed{false};
    std::mutex mu;
    auto worker = [&]() {
        try {
            for (;;) {
                if (failed.load(std::memory_order_relaxed)) return;
                int64_t b = next.fetch_add(grain);
                if (b >= n) return;
                fn(b, std::min(n, b + grain));
            }
        } catch (const std::bad_alloc &) {
            std::lock_guard<std::mutex> g(mu);
            failed = true;
            err = "host allocation failed during conversion";
        } catch (const std::exception &e) {
            std::lock_guard<std::mutex> g(mu);
            failed = true;
            err = e.what();
        }
    };
    int T = (int)std::max<int64_t>(1, std::min<int64_t>(nthreads, (n + grain - 1) / grain));
    std::vector<std::thread> th;
    for (int i = 1; i < T; ++i) th.emplace_back(worker);
    worker();
    for (auto &t : th) t.join();
    return !failed.load();
}

struct Entry {
    uint64_t key;  // chunk << 8 | local_row << 4 | local_col
    int64_t idx;   // position in the CSR arrays
};

inline int select_format(int64_t nnz, int th1, int th2) {
    if (nnz < th1) return CB_FMT_COO;  // Section 3.3.2
    if (nnz > th2) return CB_FMT_DENSE;
    return CB_FMT_CSR;
}

inline void store_value(uint8_t *dst, double v, int vtype) {
    if (vtype == CB_VALUE_F64) {
        std::memcpy(dst, &v, 8);
    } else if (vtype == CB_VALUE_F32) {
        uint32_t b = f32_bits_rne(v);
        std::memcpy(dst, &b, 4);
    } else {
        uint16_t b = bf16_bits_rne(v);
        std::memcpy(dst, &b, 2);
    }
}

struct PanelCounts {
    int64_t tiles = 0, bytes = 0, cols = 0, fmt[3] = {0, 0, 0};
    int64_t flat = 0, runs = 0;  // COO/CSR entries and (tile, row) runs
    int64_t span = 0;            // aggregation: the widest tile's original columns, last minus first
};

// Groups the entries of one panel (S = blk rows) into S x S tiles.  With
// aggregation the panel's distinct columns (ascending) are its aggregated
// columns and chunk c holds aggregated columns [S c, S c + S) (Section 3.3.1);
// without it chunk = column / S.  Entries end up row-major inside each tile.
class PanelBuilder {
  public:
    PanelBuilder(const int64_t *rp, const int32_t *ci, int64_t m, int lt) : rp_(rp), ci_(ci), m_(m), lt_(lt) {}

    void build(int64_t p, bool agg) {
        const int64_t S = (int64_t)1 << lt_;
        const int64_t r0 = p * S, r1 = std::min(m_, r0 + S);
        const int64_t e0 = rp_[r0], e1 = rp_[r1];
        cols_.clear();
        ent_.clear();
        if (agg) {
            cols_.assign(ci_ + e0, ci_ + e1);
            std::sort(cols_.begin(), cols_.end());
            cols_.erase(std::unique(cols_.begin(), cols_.end()), cols_.end());
        }
        ent_.reserve((size_t)(e1 - e0));
        for (int64_t r = r0; r < r1; ++r) {
            const uint64_t lr = (uint64_t)(r - r0);
            for (int64_t t = rp_[r]; t < rp_[r + 1]; ++t) {
                uint64_t a;
                if (agg)
                    a = (uint64_t)(std::lower_bound(cols_.begin(), cols_.end(), ci_[t]) - cols_.begin());
                else
                    a = (uint64_t)ci_[t];
                ent_.push_back({((a >> lt_) << 8) | (lr << 4) | (a & (uint64_t)(S - 1)), t});
            }
        }
        std::sort(ent_.begin(), ent_.end(), [](const Entry &x, const Entry &y) { return x.key < y.key; });
    }

    const std::vector<int32_t> &cols() const { return cols_; }
    const std::vector<Entry> &entries() const { return ent_; }

  private:
    const int64_t *rp_;
    const int32_t *ci_;
    int64_t m_;
    int lt_;  // log2 of the tile size
    std::vector<int32_t> cols_;
    std::vector<Entry> ent_;
};

template <class F>
void for_each_tile(const std::vector<Entry> &ent, F &&f) {
    size_t b = 0;
    while (b < ent.size()) {
        size_t e = b + 1;
        const uint64_t chunk = ent[b].key >> 8;
        while (e < ent.size() && (ent[e].key >> 8) == chunk) ++e;
        f((int64_t)chunk, b, e);
        b = e;
    }
}

void moments(const std::vector<int64_t> &v, int64_t &mx, double &mean, double &sd) {
    mx = 0;
    mean = sd = 0.0;
    if (v.empty()) return;
    long double s = 0, s2 = 0;
    for (int64_t x : v) {
        mx = std::max(mx, x);
        s += x;
    }
    mean = (double)(s / v.size());
    for (int64_t x : v) s2 += ((long double)x - mean) * ((long double)x - mean);
    sd = std::sqrt((double)(s2 / v.size()));
}

void build_tile_cols(HostStructure &s);
void build_tile_c16(HostStructure &s, int mode);

// Batches of the streaming kernel (format in cb_stream.h): every work range
// is cut, in order, into runs of at most kBatchTiles tiles whose payload bytes
// touch at most kRingChunks chunks of kChunk bytes and whose panels lie within
// kBatchPanels consecutive ones.
void build_stream(HostStructure &s) {
    using namespace cbs;
    const int vs = s.vsize, S = s.blk;
    const int64_t NW = s.nwaves;
    s.batch_ptr.assign((size_t)NW + 1, 0);
    std::vector<int32_t> &bs = s.batch_stream;
    bs.clear();
    int64_t nb = 0;
    auto region = [&](int64_t t) { return region_bytes(s.tile_type[t], s.tile_nnz[t], vs, S); };
    auto push = [&](int32_t a, int32_t b, int32_t c, int32_t d) {
        bs.push_back(a);
        bs.push_back(b);
        bs.push_back(c);
        bs.push_back(d);
    };
    for (int64_t w = 0; w < NW; ++w) {
        s.batch_ptr[w] = (int32_t)(bs.size() / 4);
        const int64_t t0 = s.wave_ptr[w], t1 = s.wave_ptr[w + 1];
        if (t0 >= t1) continue;
        const int64_t B0 = s.tile_vp[t0];
        int64_t b = t0;
        while (b < t1) {
            const int64_t rs = s.tile_vp[b] - B0;
            int64_t e = b + 1;
            while (e < t1 && e - b < kBatchTiles && s.tile_row[e] - s.tile_row[b] < kBatchPanels) {
                const int64_t re_e = s.tile_vp[e] - B0 + region(e);
                if (((re_e - 1) / kChunk) - rs / kChunk + 1 > kRingChunks) break;
                ++e;
            }
            const int64_t re = s.tile_vp[e - 1] - B0 + region(e - 1);
            const int32_t pb = s.tile_row[b];
            uint32_t done = 0;
            int nflat = 0, ndense = 0;
            for (int64_t t = b; t < e; ++t) {
                done |= 1u << (s.tile_row[t] - pb);
                if (s.tile_type[t] == CB_FMT_DENSE) ++ndense; else ++nflat;
            }
            if (e < t1 && s.tile_row[e] == s.tile_row[e - 1]) done &= ~(1u << (s.tile_row[e - 1] - pb));
            const size_t hdr = bs.size();
            push(0, 0, 0, 0);
            int64_t es = 0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int64_t t = b; t < e; ++t) {
                    const int fmt = s.tile_type[t];
                    if ((fmt == CB_FMT_DENSE) != (pass == 1)) continue;
                    const int64_t rel = s.tile_vp[t] - B0, nz = s.tile_nnz[t];
                    const uint32_t tag = ((uint32_t)(s.tile_row[t] & (kBatchPanels - 1)) << 24) | ((uint32_t)(t - b) << 27);
                    const int32_t xo = s.col_agg ? s.cols_offset[s.tile_row[t]] + S * s.tile_col[t] : s.tile_col[t];
                    if (fmt == CB_FMT_DENSE) {
                        push((int32_t)tag, 0, (int32_t)rel, xo);
                    } else {
                        const int64_t hb = fmt == CB_FMT_CSR ? S : 0;
                        const int64_t voff = rel + hb + nz + padding(hb + nz, vs);
                        const uint32_t pmask = (1u << kRingBits) - 1;
                        const uint32_t cpos = (uint32_t)(rel + hb - es) & pmask, vpos = (uint32_t)(voff - vs * es) & pmask;
                        push((int32_t)(tag | cpos | (vpos << kRingBits)), (int32_t)(es + nz - 1), 0, xo);
                        es += nz;
                    }
                }
            }
            bs[hdr] = (int32_t)re;
            bs[hdr + 1] = pb;
            bs[hdr + 2] = (int32_t)((e - b) | (nflat << 8) | (ndense << 16) | (done << 24));
            bs[hdr + 3] = (int32_t)es;
            ++nb;
            b = e;
        }
    }
    s.batch_ptr[NW] = (int32_t)(bs.size() / 4);
    s.nbatches = nb;
    s.nrecords = (int64_t)(bs.size() / 4);
    s.panel_tile.assign((size_t)s.npanels + 1, 0);
    {
        int64_t t = 0;
        for (int64_t p = 0; p <= s.npanels; ++p) {
            while (t < s.ntiles && s.tile_row[t] < p) ++t;
            s.panel_tile[(size_t)p] = (int32_t)t;
        }
    }
    s.tile_rec.resize((size_t)s.ntiles * 4);
    for (int64_t t = 0; t < s.ntiles; ++t) {
        const uint64_t vp = (uint64_t)s.tile_vp[t];
        s.tile_rec[(size_t)(4 * t)] = (int32_t)(uint32_t)vp;
        s.tile_rec[(size_t)(4 * t + 1)] =
            (int32_t)((uint32_t)((vp >> 32) & 0xFFFFu) | ((uint32_t)s.tile_type[t] << 16) | ((uint32_t)(s.tile_nnz[t] - 1) << 18));
        s.tile_rec[(size_t)(4 * t + 2)] = s.tile_row[t];
        s.tile_rec[(size_t)(4 * t + 3)] = s.tile_col[t];
    }
    build_tile_cols(s);
}

// Under aggregation, every tile's S original columns in kernel order (tile_cols, cb_stream.h).
void build_tile_cols(HostStructure &s) {
    const int S = s.blk;
    s.tile_cols.clear();
    if (s.col_agg) {
        s.tile_cols.resize((size_t)s.ntiles * S);
        for (int64_t t = 0; t < s.ntiles; ++t) {
            const int64_t p = s.tile_row[t], base = s.cols_offset[p] + (int64_t)S * s.tile_col[t];
            const int64_t width = std::min<int64_t>(S, s.cols_offset[p + 1] - base);
            // column c at position (c mod 4) * (S / 4) + c / 4: a lane of a matrix-core operand that
            // needs columns q, q + 4, ... reads them as one 16-byte (S = 16) or 8-byte (S = 8) load
            for (int c = 0; c < S; ++c)
                s.tile_cols[(size_t)(t * S + (c & 3) * (S / 4) + (c >> 2))] =
                    s.restore_cols[(size_t)(c < width ? base + c : s.cols_offset[p])];
        }
    }
}

// cols16: the original columns as 16-bit offsets from a base, in two forms.  Quad batches (the quad
// kernel): where every batch's columns span less than 65,536 (the block operator: a batch covers at
// most four panels, whose columns lie within one plane of the diagonal), the base is the batch's
// lowest column, kept in the batch header's fourth word, so the kernel adds one wave-uniform value
// (cols16 2: no register or load per lane).  Otherwise, where every tile's columns span less than
// 65,536 (stencils too), the base is each tile's first column, in tile_cbase (cols16 1: one more load
// and register per lane and gather).  Columns past a tile's last are offset 0; built from tile_cols,
// in the same kernel order.  Automatic (mode 0): the per-tile form not for the quad kernel with double
// vectors, whose registers are at the limit of six wavefronts per SIMD (3D block matrix FP64 155
// against 129 us; given five wavefronts, 137 against 138); elsewhere the 2-byte forms measured faster
// (192^3 Poisson, streaming kernel: FP64 148 against 159 us, FP32 108 against 118; 3D block matrix,
// quad kernel: FP32 82 against 85, BF16 70 against 73).
void build_tile_c16(HostStructure &s, int mode) {
    const int S = s.blk;
    s.cols16 = 0;
    s.tile_cbase.clear();
    s.tile_c16.clear();
    // the rows-per-lane kernel (spmv_kernel 1) reads the 4-byte columns
    if (!s.col_agg || mode < 0 || s.ntiles == 0 || s.spmv_kernel == 1) return;
    const bool quad = s.spmv_kernel == 2 || s.lb_mode == CB_LB_PAPER_STREAM;
    std::vector<int32_t> first_col((size_t)s.ntiles), last_col((size_t)s.ntiles);
    for (int64_t t = 0; t < s.ntiles; ++t) {
        const int64_t p = s.tile_row[t], first = s.cols_offset[p] + (int64_t)S * s.tile_col[t];
        const int64_t width = std::min<int64_t>(S, s.cols_offset[p + 1] - first);
        first_col[(size_t)t] = s.restore_cols[(size_t)first];
        last_col[(size_t)t] = s.restore_cols[(size_t)(first + width - 1)];
    }
    auto offsets = [&](std::vector<uint16_t> &off, auto &&base_of) {
        off.assign((size_t)s.ntiles * S, 0);
        for (int64_t t = 0; t < s.ntiles; ++t) {
            const int64_t p = s.tile_row[t], first = s.cols_offset[p] + (int64_t)S * s.tile_col[t];
            const int64_t width = std::min<int64_t>(S, s.cols_offset[p + 1] - first);
            const int64_t b = base_of(t);
            for (int c = 0; c < S; ++c)
                off[(size_t)(t * S + c)] = (uint16_t)(c < width ? (int64_t)s.restore_cols[(size_t)(first + c)] - b : 0);
        }
    };
    if (quad) {
        // the batches' spans, from the quad batch headers (tiles consecutive from each range's first)
        bool fits = true;
        std::vector<int32_t> tile_base((size_t)s.ntiles, 0);
        for (int64_t w = 0; w < s.nwaves && fits; ++w) {
            int64_t t = s.wave_ptr[w];
            for (int64_t o = s.batch_ptr[w]; o < s.batch_ptr[w + 1] && fits;) {
                const int64_t nt = s.batch_stream[(size_t)(4 * o + 1)] & 0xFF;
                int64_t lo = INT64_MAX, hi = INT64_MIN;
                for (int64_t i = t; i < t + nt; ++i) {
                    lo = std::min<int64_t>(lo, first_col[(size_t)i]);
                    hi = std::max<int64_t>(hi, last_col[(size_t)i]);
                }
                if (hi - lo > 0xFFFF) fits = false;
                for (int64_t i = t; i < t + nt; ++i) tile_base[(size_t)i] = (int32_t)lo;
                s.batch_stream[(size_t)(4 * o + 3)] = (int32_t)lo;
                t += nt;
                o += 1 + nt;
            }
        }
        if (fits) {
            offsets(s.tile_c16, [&](int64_t t) { return (int64_t)tile_base[(size_t)t]; });
            s.cols16 = 2;
            return;
        }
        for (int64_t w = 0; w < s.nwaves; ++w)  // the headers' fourth words back to 0: no batch base
            for (int64_t o = s.batch_ptr[w]; o < s.batch_ptr[w + 1]; o += 1 + (s.batch_stream[(size_t)(4 * o + 1)] & 0xFF))
                s.batch_stream[(size_t)(4 * o + 3)] = 0;
        if (mode == 0 && s.vector_f64) return;
    }
    for (int64_t t = 0; t < s.ntiles; ++t)
        if (last_col[(size_t)t] - first_col[(size_t)t] > 0xFFFF) return;  // 4-byte columns
    s.tile_cbase = first_col;
    offsets(s.tile_c16, [&](int64_t t) { return (int64_t)first_col[(size_t)t]; });
    s.cols16 = 1;
}

// Quad batches of the quad kernel (format in cb_stream.h), written to batch_stream / batch_ptr in
// place of build_stream's batches; scatter: the batches' tiles may come from any panels (Algorithm
// 2's order), each record carries its tile's panel.
void build_qstream(HostStructure &s, bool scatter) {
    using namespace cbs;
    const int vs = s.vsize, S = s.blk;
    const int64_t NW = s.nwaves;
    s.batch_ptr.assign((size_t)NW + 1, 0);
    std::vector<int32_t> &bs = s.batch_stream;
    bs.clear();
    int64_t nb = 0;
    auto quads = [&](int64_t t) -> int64_t {
        return s.tile_type[t] == CB_FMT_DENSE ? S * S / 4 : (s.tile_nnz[t] + 3) / 4;
    };
    auto push = [&](int32_t a, int32_t b, int32_t c, int32_t d) {
        bs.push_back(a);
        bs.push_back(b);
        bs.push_back(c);
        bs.push_back(d);
    };
    for (int64_t w = 0; w < NW; ++w) {
        s.batch_ptr[w] = (int32_t)(bs.size() / 4);
        const int64_t t0 = s.wave_ptr[w], t1 = s.wave_ptr[w + 1];
        if (t0 >= t1) continue;
        const int64_t B0 = s.tile_vp[t0];
        int64_t b = t0;
        while (b < t1) {
            int64_t e = b + 1, qtot = quads(b);
            while (e < t1 && e - b < kQTiles && (scatter || s.tile_row[e] - s.tile_row[b] < kBatchPanels) &&
                   qtot + quads(e) <= (int64_t)kQPasses * 64) {
                qtot += quads(e);
                ++e;
            }
            const int32_t pb = scatter ? 0 : s.tile_row[b];
            uint32_t done = 0;
            if (!scatter) {
                for (int64_t t = b; t < e; ++t) done |= 1u << (s.tile_row[t] - pb);
                if (e < t1 && s.tile_row[e] == s.tile_row[e - 1]) done &= ~(1u << (s.tile_row[e - 1] - pb));
            }
            const int64_t np = (qtot + 63) / 64;
            push(pb, (int32_t)((e - b) | (np << 8) | (done << 16)), (int32_t)qtot, 0);
            int64_t qs = 0;
            for (int64_t t = b; t < e; ++t) {
                const int fmt = s.tile_type[t];
                const int64_t rel = s.tile_vp[t] - B0, nz = s.tile_nnz[t];
                const uint32_t dense = fmt == CB_FMT_DENSE ? 1u : 0u;
                const int64_t lim = fmt == CB_FMT_DENSE ? 0 : 4 * qs + nz;
                // scatter: {.., .., panel, position in batch | qs << 5 | dense << 15 | lim << 16}
                const uint32_t meta = scatter ? (uint32_t)(t - b) | ((uint32_t)qs << 5) | (dense << 15) |
                                                    ((uint32_t)lim << 16)
                                              : (uint32_t)(s.tile_row[t] & (kBatchPanels - 1)) | ((uint32_t)qs << 2) |
                                                    (dense << 15);
                const int32_t third = scatter ? s.tile_row[t] : (int32_t)lim;
                if (fmt == CB_FMT_DENSE) {
                    push((int32_t)(rel + (int64_t)S * S * vs), (int32_t)(rel - 4 * vs * qs), third, (int32_t)meta);
                } else {
                    const int64_t hb = fmt == CB_FMT_CSR ? S : 0;
                    const int64_t crel = rel + hb, vrel = rel + hb + nz + padding(hb + nz, vs);
                    push((int32_t)(crel - 4 * qs), (int32_t)(vrel - 4 * vs * qs), third, (int32_t)meta);
                }
                qs += quads(t);
            }
            ++nb;
            b = e;
        }
    }
    s.batch_ptr[NW] = (int32_t)(bs.size() / 4);
    s.nbatches = nb;
    s.nrecords = (int64_t)(bs.size() / 4);
}

}  // namespace

int padding(int64_t index_bytes, int vsize) {
    // Algorithm 3: (nnz * size(Idx)) mod size(Val), complemented when non-zero
    const int r = (int)(index_bytes % vsize);
    return r ? vsize - r : 0;
}

int64_t region_bytes(int fmt, int64_t nnz, int vsize, int blk) {
    int64_t b;
    if (fmt == CB_FMT_COO)
        b = nnz + padding(nnz, vsize) + nnz * vsize;
    else if (fmt == CB_FMT_CSR)
        b = blk + nnz + padding(blk + nnz, vsize) + nnz * vsize;
    else
        b = (int64_t)blk * blk * vsize + dense_mask_bytes(blk);
    return (b + kTileAlign - 1) / kTileAlign * kTileAlign;
}

uint32_t f32_bits_rne(double v) {
    // the FP64 -> FP32 conversion of the host FPU in its default
    // round-to-nearest-even mode; NaN payloads keep their top bits, quiet
    const float f = (float)v;
    uint32_t b;
    std::memcpy(&b, &f, 4);
    return b;
}

uint16_t bf16_bits_rne(double v) {
    // Round-to-odd to FP32 followed by round-to-nearest-even to BF16 equals a
    // single RNE rounding from FP64 (Boldo and Melquiond, "Emulation of FMA
    // and correctly rounded sums: proved algorithms using rounding to odd",
    // IEEE TC 2008): FP32 keeps 16 more significand bits than BF16.
    if (std::isnan(v)) return (uint16_t)((f32_bits_rne(v) >> 16) | 0x0040u);
    const float f = (float)v;
    uint32_t b;
    std::memcpy(&b, &f, 4);
    if (std::isfinite(f) && (double)f != v) {
        if (std::fabs((double)f) > std::fabs(v)) b -= 1u;  // step back to the truncated value
        b |= 1u;                                           // sticky bit: round to odd
    }
    if ((b & 0x7F800000u) == 0x7F800000u) return (uint16_t)(b >> 16);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

cb_status_t convert(int64_t m, int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                    const double *values, const cb_options_t &opt, HostStructure &out, std::string &err,
                    int64_t max_range_span) {
    const auto t_start = std::chrono::steady_clock::now();
    const int64_t kLim = (int64_t)1 << 31;
    if (m < 0 || n < 0 || nnz < 0) { err = "negative size"; return CB_ERROR_INVALID_VALUE; }
    if (m >= kLim || n >= kLim || nnz >= kLim) { err = "m, n and nnz must be below 2^31"; return CB_ERROR_INVALID_VALUE; }
    if (!row_ptr && !(m == 0 && nnz == 0)) { err = "row_ptr is NULL"; return CB_ERROR_INVALID_VALUE; }
    if (nnz > 0 && (!col_idx || !values)) { err = "col_idx or values is NULL"; return CB_ERROR_INVALID_VALUE; }
    if (opt.value_type < 0 || opt.value_type > 2) { err = "value_type out of range"; return CB_ERROR_INVALID_VALUE; }
    if (opt.col_agg < -1 || opt.col_agg > 1) { err = "col_agg must be -1, 0 or 1"; return CB_ERROR_INVALID_VALUE; }
    if (opt.th1 < 0 || opt.th2 < 0) { err = "th1 and th2 must be non-negative"; return CB_ERROR_INVALID_VALUE; }
    if (opt.quantum_tiles < 1 || opt.quantum_tiles > (1 << 20)) { err = "quantum_tiles out of range"; return CB_ERROR_INVALID_VALUE; }
    if (opt.lb_mode < 0 || opt.lb_mode > 3) { err = "lb_mode out of range"; return CB_ERROR_INVALID_VALUE; }
    if (opt.wave_nnz < 0) { err = "wave_nnz must be non-negative"; return CB_ERROR_INVALID_VALUE; }
    if (opt.min_wave_nnz < 0) { err = "min_wave_nnz must be non-negative"; return CB_ERROR_INVALID_VALUE; }
    if (opt.row_reduce < -1 || opt.row_reduce > 4) { err = "row_reduce must be -1 .. 4"; return CB_ERROR_INVALID_VALUE; }
    if (opt.vector_f64 < 0 || opt.vector_f64 > 1) { err = "vector_f64 must be 0 or 1"; return CB_ERROR_INVALID_VALUE; }
    if (opt.spmv_kernel < -1 || opt.spmv_kernel > 2) { err = "spmv_kernel must be -1, 0, 1 or 2"; return CB_ERROR_INVALID_VALUE; }
    if (opt.xcd_chunk < -1 || opt.xcd_chunk > (1 << 20)) { err = "xcd_chunk must be -1 .. 2^20"; return CB_ERROR_INVALID_VALUE; }
    if (opt.cols16 < -1 || opt.cols16 > 1) { err = "cols16 must be -1, 0 or 1"; return CB_ERROR_INVALID_VALUE; }
    if (opt.tile_dim != 0 && opt.tile_dim != 8 && opt.tile_dim != 16) { err = "tile_dim must be 0, 8 or 16"; return CB_ERROR_INVALID_VALUE; }
    if (opt.lb_mode == CB_LB_PAPER_STREAM && (opt.tile_dim == 8 || (opt.spmv_kernel >= 0 && opt.spmv_kernel != 2))) {
        err = "the streamed Algorithm 2 order runs the quad kernel on 16 x 16 tiles";
        return CB_ERROR_NOT_SUPPORTED;
    }
    if ((opt.spmv_kernel == 2 || opt.lb_mode == CB_LB_PAPER_STREAM) && n > kQuadMaxCols) {
        err = "the quad kernel (spmv_kernel 2, lb_mode paper_stream) takes at most 2^29 - 16 columns";
        return CB_ERROR_NOT_SUPPORTED;
    }
    if (opt.tile_dim == 8 && opt.spmv_kernel == 1) {
        err = "the rows-per-lane kernel (spmv_kernel 1) takes 16 x 16 tiles only";
        return CB_ERROR_NOT_SUPPORTED;
    }
    if (std::isnan(opt.th0)) { err = "th0 is NaN"; return CB_ERROR_INVALID_VALUE; }
    const int nth = opt.host_threads > 0 ? opt.host_threads : default_threads();

    // ---- validation: canonical CSR ------------------------------------------
    if (m == 0 && nnz != 0) { err = "nnz must be 0 when m == 0"; return CB_ERROR_INVALID_VALUE; }
    if (row_ptr) {
        if (row_ptr[0] != 0) { err = "row_ptr[0] must be 0"; return CB_ERROR_INVALID_VALUE; }
        if (row_ptr[m] != nnz) { err = "row_ptr[m] must equal nnz"; return CB_ERROR_INVALID_VALUE; }
        for (int64_t i = 0; i < m; ++i)
            if (row_ptr[i + 1] < row_ptr[i]) {
                err = "row_ptr decreases at row " + std::to_string(i);
                return CB_ERROR_INVALID_VALUE;
            }
    }
    std::atomic<int64_t> bad_row{INT64_MAX};
    std::string perr;
    if (!parallel_dynamic(nth, m, 4096, [&](int64_t b, int64_t e) {
            for (int64_t i = b; i < e; ++i) {
                for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
                    const int32_t c = col_idx[t];
                    if (c < 0 || c >= n || (t > row_ptr[i] && c <= col_idx[t - 1])) {
                        int64_t cur = bad_row.load();
                        while (i < cur && !bad_row.compare_exchange_weak(cur, i)) {}
                        break;
                    }
                }
            }
        }, perr)) { err = perr; return CB_ERROR_OUT_OF_MEMORY; }
    if (bad_row.load() != INT64_MAX) {
        err = "row " + std::to_string(bad_row.load()) +
              ": column indices must lie in [0, n) and increase strictly within a row";
        return CB_ERROR_INVALID_VALUE;
    }

    HostStructure s;
    s.m = m;
    s.n = n;
    s.nnz = nnz;
    s.vtype = opt.value_type;
    s.vector_f64 = opt.value_type == CB_VALUE_F64 || opt.vector_f64 ? 1 : 0;
    s.spmv_kernel = opt.spmv_kernel > 0 ? opt.spmv_kernel : 0;
    s.xcd_chunk = opt.xcd_chunk >= 0 ? opt.xcd_chunk : 0;
    s.vsize = opt.value_type == CB_VALUE_F64 ? 8 : (opt.value_type == CB_VALUE_F32 ? 4 : 2);
    s.lb_mode = opt.lb_mode;
    s.quantum_tiles = opt.quantum_tiles;
    s.blk = opt.tile_dim == 8 ? 8 : kBlk;
    s.lt = s.blk == 8 ? 3 : 4;
    const int S = s.blk, LT = s.lt;
    const int64_t P = (m + S - 1) / S;
    s.npanels = P;

    try {
        // ---- Section 3.1 + 3.3.1: plain partition census, th0 decision ------
        // (always on the 16 x 16 partition: the paper defines super-sparse sub-blocks there)
        const int64_t P16 = (m + kBlk - 1) / kBlk;
        std::vector<int64_t> plain_cnt(P16, 0), super_cnt(P16, 0), far_cnt(P16, 0);
        const int64_t far = std::max<int64_t>(1, n / 8);  // entries this far from the diagonal: "far"
        if (!parallel_dynamic(nth, P16, 64, [&](int64_t b, int64_t e) {
                std::vector<int32_t> cb;
                for (int64_t p = b; p < e; ++p) {
                    const int64_t r0 = p * kBlk, r1 = std::min(m, r0 + kBlk);
                    cb.clear();
                    for (int64_t r = r0; r < r1; ++r)
                        for (int64_t t = row_ptr[r]; t < row_ptr[r + 1]; ++t)
                            far_cnt[p] += std::llabs((int64_t)col_idx[t] - r) > far;
                    for (int64_t t = row_ptr[r0]; t < row_ptr[r1]; ++t) cb.push_back(col_idx[t] >> 4);
                    std::sort(cb.begin(), cb.end());
                    size_t i = 0;
                    while (i < cb.size()) {
                        size_t j = i;
                        while (j < cb.size() && cb[j] == cb[i]) ++j;
                        plain_cnt[p] += 1;
                        if (j - i < (size_t)kSuperSparse) super_cnt[p] += 1;
                        i = j;
                    }
                }
            }, err)) return CB_ERROR_OUT_OF_MEMORY;
        const int64_t plain = std::accumulate(plain_cnt.begin(), plain_cnt.end(), (int64_t)0);
        const int64_t super = std::accumulate(super_cnt.begin(), super_cnt.end(), (int64_t)0);
        s.plain_tiles = plain;
        s.share = plain ? (double)super / (double)plain : 0.0;
        // workgroup-to-range mapping (measured on gfx950): the XCDs side by side in runs of 16 ranges
        // keep x lines that distant rows share (stencil and block neighbours 10^4-10^5 rows apart) in
        // every L2 between their uses (3D block matrix 142 against 148 us, 192^3 Poisson 162 against
        // 176); where many entries lie far from the diagonal (scattered columns) each XCD on its own
        // eighth keeps a narrower window of near-diagonal x instead (power-law rows 584 against 637)
        if (opt.xcd_chunk < 0) {
            const int64_t nfar = std::accumulate(far_cnt.begin(), far_cnt.end(), (int64_t)0);
            s.xcd_chunk = nfar * 20 >= nnz && nnz > 0 ? 0 : 16;
        }
        bool agg;
        if (opt.col_agg == 0) agg = false;
        else if (opt.col_agg == 1) agg = true;
        else agg = s.share >= opt.th0;  // aggregation skipped when the super-sparse share is low
        s.col_agg = agg ? 1 : 0;

        // ---- pass A: tiles, bytes and aggregated columns per panel ----------
        std::vector<PanelCounts> pc(P);
        if (!parallel_dynamic(nth, P, 64, [&](int64_t b, int64_t e) {
                PanelBuilder pb(row_ptr, col_idx, m, LT);
                for (int64_t p = b; p < e; ++p) {
                    pb.build(p, agg);
                    PanelCounts c;
                    c.cols = agg ? (int64_t)pb.cols().size() : 0;
                    if (agg)
                        for (size_t i = 0; i < pb.cols().size(); i += S)
                            c.span = std::max<int64_t>(c.span, (int64_t)pb.cols()[std::min(i + S, pb.cols().size()) - 1] -
                                                                   pb.cols()[i]);
                    const std::vector<Entry> &ent = pb.entries();
                    for_each_tile(ent, [&](int64_t, size_t lo, size_t hi) {
                        const int fmt = select_format((int64_t)(hi - lo), opt.th1, opt.th2);
                        c.tiles += 1;
                        c.fmt[fmt] += 1;
                        c.bytes += region_bytes(fmt, (int64_t)(hi - lo), s.vsize, S);
                        if (fmt != CB_FMT_DENSE) {
                            c.flat += (int64_t)(hi - lo);
                            for (size_t i = lo; i < hi; ++i) c.runs += (i == lo || (ent[i].key >> 4) != (ent[i - 1].key >> 4));
                        }
                    });
                    pc[p] = c;
                }
            }, err)) return CB_ERROR_OUT_OF_MEMORY;

        std::vector<int64_t> tile_base(P + 1, 0), byte_base(P + 1, 0), col_base(P + 1, 0);
        int64_t span = 0;
        for (int64_t p = 0; p < P; ++p) {
            span = std::max(span, pc[p].span);
            tile_base[p + 1] = tile_base[p] + pc[p].tiles;
            byte_base[p + 1] = byte_base[p] + pc[p].bytes;
            col_base[p + 1] = col_base[p] + pc[p].cols;
            for (int f = 0; f < 3; ++f) s.tiles_fmt[f] += pc[p].fmt[f];
            s.flat_entries += pc[p].flat;
            s.flat_runs += pc[p].runs;
        }
        const int64_t NT = tile_base[P];
        s.ntiles = NT;
        // row sums of the streaming kernel (measured on gfx950): FP64 LDS atomics beat the
        // segmented scan on every workload tried, FP32 LDS atomics lose to it on every one, so
        // FP32/BF16 products are summed with FP64 atomics too; where a tile row's entries come in
        // runs of two or more (dense blocks) the two accumulator copies halve the collisions on one
        // address (3D block matrix: 3.5 % faster in FP64, 12 % in FP32), where they come one by one
        // (stencils, scattered rows) the copies only cost LDS
        // natural-order kernel (measured on gfx950): the quad kernel wins where tiles are well filled
        // and their rows hold runs of entries (3D block matrix: FP64 147 against 153 us, BF16 77 against
        // 105), the streaming kernel where tiles are sparse or rows come one entry per tile row
        // (stencils, power-law rows), whose quads are part empty and sum no runs -- except with float
        // vectors where 2-byte column offsets apply (cols16): there the quad kernel won on the 192^3
        // Poisson operator too (FP32 105.9 against 108.8 us, BF16 92.1 against 102.5)
        if (opt.spmv_kernel < 0 && natural_lb(s.lb_mode)) {
            const bool long_runs = s.flat_runs > 0 && s.flat_entries >= 2 * s.flat_runs;
            const bool float_c16 = !s.vector_f64 && agg && opt.cols16 >= 0 && span <= 0xFFFF;
            s.spmv_kernel = ((long_runs && nnz >= 32 * NT) || float_c16) && n <= kQuadMaxCols ? 2 : 0;
        }
        if (s.lb_mode == CB_LB_PAPER_STREAM) s.spmv_kernel = 2;  // the quad kernel's scatter form
        if (opt.row_reduce >= 0) {
            s.row_reduce = opt.row_reduce;
            // the quad kernel sums each lane's row runs in registers instead of a segmented scan
            if (s.spmv_kernel == 2 && s.row_reduce == 1) s.row_reduce = 0;
        } else {
            // the quad kernel sums a lane's row runs in registers before its one LDS add, so one
            // copy of the row sums serves it (3D block matrix: FP64 131.0 against 132.4 us with two,
            // FP32 83.6 against 84.2, BF16 within noise)
            const bool runs = s.flat_runs > 0 && s.flat_entries >= 2 * s.flat_runs && s.spmv_kernel != 2;
            if (s.vector_f64) s.row_reduce = runs ? 3 : 0;
            else s.row_reduce = runs ? 4 : 2;
        }
        if (NT >= kLim || col_base[P] >= kLim) { err = "structure too large"; return CB_ERROR_NOT_SUPPORTED; }

        // natural-order arrays and the packed payload (Section 3.2)
        std::vector<int32_t> nrow(NT), ncol(NT), nnzv(NT);
        std::vector<int64_t> nvp(NT);
        std::vector<uint8_t> ntype(NT);
        s.payload.assign((size_t)byte_base[P], 0);
        if (agg) {
            s.restore_cols.resize((size_t)col_base[P]);
            s.cols_offset.resize((size_t)P + 1);
            for (int64_t p = 0; p <= P; ++p) s.cols_offset[p] = (int32_t)col_base[p];
        }

        // ---- pass B: write tiles --------------------------------------------
        const int vs = s.vsize, vt = s.vtype;
        if (!parallel_dynamic(nth, P, 64, [&](int64_t b, int64_t e) {
                PanelBuilder pb(row_ptr, col_idx, m, LT);
                for (int64_t p = b; p < e; ++p) {
                    pb.build(p, agg);
                    if (agg) std::copy(pb.cols().begin(), pb.cols().end(), s.restore_cols.begin() + col_base[p]);
                    int64_t ti = tile_base[p], off = byte_base[p];
                    const auto &ent = pb.entries();
                    for_each_tile(ent, [&](int64_t chunk, size_t lo, size_t hi) {
                        const int64_t nz = (int64_t)(hi - lo);
                        const int fmt = select_format(nz, opt.th1, opt.th2);
                        nrow[ti] = (int32_t)p;
                        ncol[ti] = (int32_t)chunk;
                        nnzv[ti] = (int32_t)nz;
                        nvp[ti] = off;
                        ntype[ti] = (uint8_t)fmt;
                        uint8_t *base = s.payload.data() + off;
                        if (fmt == CB_FMT_DENSE) {
                            uint8_t *mask = base + (int64_t)S * S * vs;
                            for (size_t q = lo; q < hi; ++q) {
                                // element (lr, lc) of the S x S tile, row-major
                                const int slot = (int)(((ent[q].key >> 4) & 15u) * (uint64_t)S + (ent[q].key & 15u));
                                store_value(base + (int64_t)slot * vs, values[ent[q].idx], vt);
                                mask[slot >> 3] |= (uint8_t)(1u << (slot & 7));
                            }
                        } else {
                            uint8_t *codes = base;
                            int64_t hdr = 0;
                            if (fmt == CB_FMT_CSR) {
                                hdr = S;
                                codes = base + S;
                                // one-byte row starts: entries before row r
                                int cnt[kBlk + 1] = {0};
                                for (size_t q = lo; q < hi; ++q) cnt[((ent[q].key >> 4) & 15u) + 1] += 1;
                                for (int r = 0; r < S; ++r) {
                                    cnt[r + 1] += cnt[r];
                                    base[r] = (uint8_t)cnt[r];
                                }
                            }
                            uint8_t *vals = codes + nz + padding(hdr + nz, vs);
                            for (size_t q = lo; q < hi; ++q) {
                                const uint32_t lr = (uint32_t)((ent[q].key >> 4) & 15u), lc = (uint32_t)(ent[q].key & 15u);
                                codes[q - lo] = (uint8_t)((lc << 4) | lr);  // Algorithm 3: row = b & 15, col = b >> 4
                                store_value(vals + (int64_t)(q - lo) * vs, values[ent[q].idx], vt);
                            }
                        }
                        off += region_bytes(fmt, nz, vs, S);
                        ++ti;
                    });
                }
            }, err)) return CB_ERROR_OUT_OF_MEMORY;

        // ---- Section 3.4: grouping into work units ---------------------------
        const int W = opt.quantum_tiles;
        std::vector<int32_t> order(NT);
        std::vector<int32_t> qptr;
        if (opt.lb_mode == CB_LB_PAPER || opt.lb_mode == CB_LB_PAPER_STREAM) {
            // Algorithm 2: descending nnz (stable), min-heap of (load, tb_id), W slots per block
            std::vector<int32_t> byn(NT);
            std::iota(byn.begin(), byn.end(), 0);
            std::stable_sort(byn.begin(), byn.end(), [&](int32_t a, int32_t b) { return nnzv[a] > nnzv[b]; });
            const int64_t T = (NT + W - 1) / W;
            struct Slot {
                int64_t load;
                int64_t tb;
                int32_t warps;
            };
            auto cmp = [](const Slot &a, const Slot &b) { return a.load != b.load ? a.load > b.load : a.tb > b.tb; };
            std::priority_queue<Slot, std::vector<Slot>, decltype(cmp)> pq(cmp);
            for (int64_t tb = 0; tb < T; ++tb) pq.push({0, tb, 0});
            std::vector<int32_t> slot((size_t)(T * W), -1);
            for (int64_t i = 0; i < NT; ++i) {
                Slot top = pq.top();
                pq.pop();
                const int32_t blk = byn[i];
                slot[(size_t)(top.tb * W + top.warps)] = blk;  // end = tb_id * W + warps
                top.load += nnzv[blk];
                top.warps += 1;
                if (top.warps < W) pq.push(top);
            }
            // sort by end = keep slot order, dropping the empty slots but not the group boundaries
            qptr.assign((size_t)T + 1, 0);
            int64_t k = 0;
            for (int64_t tb = 0; tb < T; ++tb) {
                for (int w = 0; w < W; ++w) {
                    const int32_t blk = slot[(size_t)(tb * W + w)];
                    if (blk >= 0) order[k++] = blk;
                }
                qptr[tb + 1] = (int32_t)k;
            }
        } else {
            std::iota(order.begin(), order.end(), 0);
            if (opt.lb_mode == CB_LB_NONE) {
                const int64_t T = (NT + W - 1) / W;
                qptr.assign((size_t)T + 1, 0);
                for (int64_t tb = 0; tb <= T; ++tb) qptr[tb] = (int32_t)std::min<int64_t>(NT, tb * W);
            }
        }

        // target work per wavefront range, in non-zero equivalents
        const int64_t total_w = nnz + (int64_t)kTileCost * NT;
        int64_t target = opt.wave_nnz;
        bool taper = false;
        if (target == 0) {
            const int64_t cap = std::min<int64_t>(4096, CB_TUNE_MAX_RANGE_BYTES / (1 + s.vsize));
            const int64_t floor_w = std::max<int64_t>(CB_TUNE_MIN_WAVE_NNZ, opt.min_wave_nnz);
            target = std::min<int64_t>(std::max(cap, floor_w),
                                       std::max<int64_t>(floor_w, (total_w + CB_TUNE_WAVE_RANGES - 1) / CB_TUNE_WAVE_RANGES));
            // not under the eighths mapping: it deals the XCDs equal counts of ranges, and shorter
            // ranges at the end would leave the last XCD less work (power-law rows 626 against 584 us)
            taper = target == cap && s.xcd_chunk != 0;
        }
        auto tw = [&](int32_t i) { return (int64_t)nnzv[i] + kTileCost; };

        std::vector<int32_t> wptr;
        if (opt.lb_mode == CB_LB_CONTIGUOUS) {
            // natural order cut at panel boundaries; a panel heavier than twice
            // the target is cut at tile boundaries into pieces of about the target
            wptr.push_back(0);
            int64_t cur = 0;
            int64_t rem = total_w;
            const int64_t full_target = target;
            for (int64_t p = 0; p < P; ++p) {
                const int64_t b = tile_base[p], e = tile_base[p + 1];
                if (b == e) continue;
                int64_t wp = 0;
                for (int64_t i = b; i < e; ++i) wp += tw((int32_t)i);
                if (taper)
                    target = std::min(full_target, std::max(std::max<int64_t>(CB_TUNE_MIN_WAVE_NNZ, full_target / CB_TUNE_TAPER_FLOOR),
                                                            rem / CB_TUNE_TAPER_DIV));
                rem -= wp;
                if (wp > 2 * target) {
                    if (cur > 0) { wptr.push_back((int32_t)b); cur = 0; }
                    const int64_t pieces = (wp + target - 1) / target;
                    const int64_t piece_w = (wp + pieces - 1) / pieces;
                    int64_t acc = 0;
                    for (int64_t i = b; i < e; ++i) {
                        acc += tw((int32_t)i);
                        if (acc >= piece_w && i + 1 < e) { wptr.push_back((int32_t)(i + 1)); acc = 0; }
                    }
                    wptr.push_back((int32_t)e);
                    cur = 0;
                } else {
                    if (cur > 0 && cur + wp > target) { wptr.push_back((int32_t)b); cur = 0; }
                    cur += wp;
                }
            }
            if (wptr.back() != (int32_t)NT) wptr.push_back((int32_t)NT);
            if (NT == 0) wptr.assign(1, 0);
            qptr = wptr;
            target = full_target;
        } else {
            const int64_t T = (int64_t)qptr.size() - 1;
            const double mean_q = T > 0 ? (double)total_w / (double)T : 1.0;
            const int64_t G = std::max<int64_t>(1, (int64_t)std::llround((double)target / std::max(1.0, mean_q)));
            for (int64_t q = 0; q < T; q += G) wptr.push_back(qptr[q]);
            wptr.push_back((int32_t)NT);
            if (NT == 0) wptr.assign(1, 0);
        }

        // ---- kernel-order arrays --------------------------------------------
        s.tile_row.resize(NT);
        s.tile_col.resize(NT);
        s.tile_nnz.resize(NT);
        s.tile_vp.resize(NT);
        s.tile_type.resize(NT);
        s.tile_ori = order;
        for (int64_t i = 0; i < NT; ++i) {
            const int32_t o = order[i];
            s.tile_row[i] = nrow[o];
            s.tile_col[i] = ncol[o];
            s.tile_nnz[i] = nnzv[o];
            s.tile_vp[i] = nvp[o];
            s.tile_type[i] = ntype[o];
        }
        if (agg) {
            s.tile_xoff.resize(NT);
            for (int64_t i = 0; i < NT; ++i) s.tile_xoff[i] = s.cols_offset[s.tile_row[i]] + S * s.tile_col[i];
        }
        s.quantum_ptr = qptr;
        s.wave_ptr = wptr;
        if (opt.lb_mode == CB_LB_PAPER_STREAM) {
            // the packed tiles re-laid in kernel (group) order: a work range is one byte range
            std::vector<uint8_t> repacked(s.payload.size());
            int64_t at = 0;
            for (int64_t i = 0; i < NT; ++i) {
                const int64_t rb = region_bytes(s.tile_type[i], s.tile_nnz[i], s.vsize, S);
                std::memcpy(repacked.data() + at, s.payload.data() + s.tile_vp[i], (size_t)rb);
                s.tile_vp[i] = at;
                at += rb;
            }
            s.payload.swap(repacked);
        }

        // a panel is owned when its tiles form one run inside one work range;
        // otherwise it is shared (atomics after a y <- beta*y pre-pass); empty
        // panels are written by the pre-pass alone
        std::vector<int32_t> runs(P, 0);
        const int64_t NW = (int64_t)wptr.size() - 1;
        for (int64_t w = 0; w < NW; ++w)
            for (int64_t i = wptr[w]; i < wptr[w + 1]; ++i)
                if (i == wptr[w] || s.tile_row[i] != s.tile_row[i - 1]) runs[s.tile_row[i]] += 1;
        s.panel_shared.assign(P, 0);
        for (int64_t p = 0; p < P; ++p) {
            // the scatter form adds every tile's rows with atomics: every panel is shared
            const bool scatter = opt.lb_mode == CB_LB_PAPER_STREAM;
            if (runs[p] > 1 || (scatter && runs[p] > 0)) { s.panel_shared[p] = 1; s.nshared += 1; }
            if (runs[p] != 1 || scatter) s.prepass_list.push_back((int32_t)p);
        }

        // ---- statistics -------------------------------------------------------
        std::vector<int64_t> qn, wn;
        for (size_t q = 0; q + 1 < qptr.size(); ++q) {
            int64_t a = 0;
            for (int32_t i = qptr[q]; i < qptr[q + 1]; ++i) a += s.tile_nnz[i];
            qn.push_back(a);
        }
        for (int64_t w = 0; w < NW; ++w) {
            int64_t a = 0;
            for (int32_t i = wptr[w]; i < wptr[w + 1]; ++i) a += s.tile_nnz[i];
            wn.push_back(a);
        }
        moments(qn, s.quantum_nnz_max, s.quantum_nnz_mean, s.quantum_nnz_std);
        moments(wn, s.wave_nnz_max, s.wave_nnz_mean, s.wave_nnz_std);
        s.payload_bytes = (int64_t)s.payload.size();
        s.nrestore = (int64_t)s.restore_cols.size();
        s.nquanta = (int64_t)qptr.size() - 1;
        s.nwaves = NW;
        s.nprepass = (int64_t)s.prepass_list.size();
        if (streamed_lb(opt.lb_mode)) {
            // the records' 32-bit fields bound what one range and the whole stream may hold
            if (NT + (int64_t)NW + 1 > (int64_t)INT32_MAX / 2) {
                err = "too many tiles for the streaming kernel's batch records";
                return CB_ERROR_NOT_SUPPORTED;
            }
            if (s.payload_bytes >= ((int64_t)1 << 48)) {
                err = "payload too large for the tile records";
                return CB_ERROR_NOT_SUPPORTED;
            }
            // a range's batch ends and region starts are 32-bit offsets from its first payload byte
            for (int64_t w = 0; w < NW; ++w) {
                const int64_t t0 = wptr[w], t1 = wptr[w + 1];
                if (t0 >= t1) continue;
                const int64_t span = s.tile_vp[t1 - 1] + region_bytes(s.tile_type[t1 - 1], s.tile_nnz[t1 - 1], s.vsize, S) -
                                     s.tile_vp[t0];
                if (span > max_range_span) {
                    err = "wave_nnz too large: work range " + std::to_string(w) + " would span " + std::to_string(span) +
                          " payload bytes (at most " + std::to_string(max_range_span) + ")";
                    return CB_ERROR_INVALID_VALUE;
                }
            }
            if (opt.lb_mode == CB_LB_PAPER_STREAM) {
                build_tile_cols(s);
                build_qstream(s, true);
            } else {
                build_stream(s);
                if (s.spmv_kernel == 2) build_qstream(s, false);
            }
            build_tile_c16(s, opt.cols16);
        }
    } catch (const std::bad_alloc &) {
        err = "host allocation failed during conversion";
        return CB_ERROR_OUT_OF_MEMORY;
    }
    s.convert_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    out = std::move(s);
    return CB_SUCCESS;
}

cb_status_t export_csr(const HostStructure &s, int64_t *row_ptr, int32_t *col_idx, void *values, std::string &err) {
    if (!row_ptr || (s.nnz > 0 && (!col_idx || !values))) {
        err = "NULL output buffer";
        return CB_ERROR_INVALID_VALUE;
    }
    const int vs = s.vsize, S = s.blk;
    try {
        // decode every tile into (row, col, value bits); tiles may come in any order
        std::vector<int64_t> cnt((size_t)s.m + 1, 0);
        auto visit = [&](auto &&emit) {
            for (int64_t i = 0; i < s.ntiles; ++i) {
                const int64_t p = s.tile_row[i], c = s.tile_col[i], nz = s.tile_nnz[i];
                const int fmt = s.tile_type[i];
                const uint8_t *base = s.payload.data() + s.tile_vp[i];
                auto orig_col = [&](int lc) -> int64_t {
                    if (s.col_agg) return s.restore_cols[(size_t)(s.cols_offset[p] + S * c + lc)];
                    return S * c + lc;
                };
                if (fmt == CB_FMT_DENSE) {
                    const uint8_t *mask = base + (int64_t)S * S * vs;
                    for (int e = 0; e < S * S; ++e)
                        if ((mask[e >> 3] >> (e & 7)) & 1) emit(S * p + e / S, orig_col(e % S), base + (int64_t)e * vs);
                } else {
                    const int64_t hdr = fmt == CB_FMT_CSR ? S : 0;
                    const uint8_t *codes = base + hdr;
                    const uint8_t *vals = codes + nz + padding(hdr + nz, vs);
                    for (int64_t q = 0; q < nz; ++q)
                        emit(S * p + (codes[q] & 15), orig_col(codes[q] >> 4), vals + q * vs);
                }
            }
        };
        int64_t total = 0;
        bool bad = false;
        visit([&](int64_t r, int64_t, const uint8_t *) {
            if (r < 0 || r >= s.m) { bad = true; return; }
            cnt[(size_t)r + 1] += 1;
            ++total;
        });
        if (bad || total != s.nnz) {
            err = "stored structure is inconsistent";
            return CB_ERROR_INTERNAL;
        }
        for (int64_t r = 0; r < s.m; ++r) cnt[r + 1] += cnt[r];
        std::vector<int64_t> cur(cnt.begin(), cnt.end() - 1);
        std::vector<std::pair<int32_t, uint64_t>> tmp((size_t)s.nnz);
        visit([&](int64_t r, int64_t col, const uint8_t *v) {
            uint64_t bits = 0;
            std::memcpy(&bits, v, vs);
            tmp[(size_t)cur[r]++] = {(int32_t)col, bits};
        });
        for (int64_t r = 0; r < s.m; ++r) {
            std::sort(tmp.begin() + cnt[r], tmp.begin() + cnt[r + 1],
                      [](const auto &a, const auto &b) { return a.first < b.first; });
            row_ptr[r] = cnt[r];
        }
        if (s.m >= 0) row_ptr[s.m] = s.nnz;
        uint8_t *vout = (uint8_t *)values;
        for (int64_t t = 0; t < s.nnz; ++t) {
            col_idx[t] = tmp[(size_t)t].first;
            std::memcpy(vout + t * vs, &tmp[(size_t)t].second, vs);
        }
    } catch (const std::bad_alloc &) {
        err = "host allocation failed during export";
        return CB_ERROR_OUT_OF_MEMORY;
    }
    return CB_SUCCESS;
}

int64_t spmv_bytes(const HostStructure &s) {
    const int64_t xe = s.vector_f64 ? 8 : 4;
    int64_t b = s.payload_bytes + xe * s.n + xe * s.m;  // payload, x read once, y written once
    if (s.lb_mode == CB_LB_PAPER) {
        // tile-at-a-time kernel: high-level arrays (4+4+4+8+1 per tile), restore_cols through
        // cols_offset, work ranges, panel flags, pre-pass list
        b += 21 * s.ntiles;
        if (s.col_agg) b += 4 * s.nrestore + 4 * (s.npanels + 1);
        b += 4 * (s.nwaves + 1) + s.npanels + 4 * s.nprepass;
    } else {
        // streaming kernel: batch records, 16 original columns per tile under aggregation (else one
        // column block per tile), two range pointers per range and the first tile's offset and the end
        // panels' flags, pre-pass list
        b += 16 * s.nrecords;
        b += s.col_agg ? (s.cols16 == 2 ? 2 * (int64_t)s.blk : s.cols16 ? 2 * (int64_t)s.blk + 4 : 4 * (int64_t)s.blk) * s.ntiles
                       : 4 * s.ntiles;
        b += 8 * (s.nwaves + 1) + 18 * s.nwaves + 4 * s.nprepass;
        // scatter form: the pre-pass writes y, the atomics read and write it again
        if (s.lb_mode == CB_LB_PAPER_STREAM) b += 2 * xe * s.m;
    }
    return b;
}

void fill_info(const HostStructure &s, cb_info_t &info) {
    info.value_type = s.vtype;
    info.m = s.m;
    info.n = s.n;
    info.nnz = s.nnz;
    info.npanels = s.npanels;
    info.ntiles = s.ntiles;
    info.tiles_coo = s.tiles_fmt[0];
    info.tiles_csr = s.tiles_fmt[1];
    info.tiles_dense = s.tiles_fmt[2];
    info.col_agg = s.col_agg;
    info.lb_mode = s.lb_mode;
    info.super_sparse_share = s.share;
    info.plain_tiles = s.plain_tiles;
    info.payload_bytes = s.payload_bytes;
    info.meta_bytes = 21 * s.ntiles;
    info.restore_bytes = s.col_agg ? 4 * s.nrestore + 4 * (s.npanels + 1) + 4 * s.ntiles : 0;
    info.sched_bytes = 4 * (s.nwaves + 1) + s.npanels + 4 * s.nprepass;
    info.nquanta = s.nquanta;
    info.nwaves = s.nwaves;
    info.shared_panels = s.nshared;
    info.prepass_panels = s.nprepass;
    info.quantum_nnz_max = s.quantum_nnz_max;
    info.quantum_nnz_mean = s.quantum_nnz_mean;
    info.quantum_nnz_std = s.quantum_nnz_std;
    info.wave_nnz_max = s.wave_nnz_max;
    info.wave_nnz_mean = s.wave_nnz_mean;
    info.wave_nnz_std = s.wave_nnz_std;
    info.spmv_bytes = spmv_bytes(s);
    info.nbatches = s.nbatches;
    info.stream_bytes = 16 * s.nrecords;
    info.convert_seconds = s.convert_seconds;
    info.flat_run_mean = s.flat_runs ? (double)s.flat_entries / (double)s.flat_runs : 0.0;
    info.row_reduce = s.row_reduce;
    info.vector_f64 = s.vector_f64;
    info.spmv_kernel = s.spmv_kernel;
    info.xcd_chunk = s.xcd_chunk;
    info.cols16 = s.cols16;
    info.tile_dim = s.blk;
}

}  // namespace cbh
