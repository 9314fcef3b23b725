"""Host-side checks of the streaming kernel's batch records (no GPU).

The converter cuts every work range into batches and writes a header and one
record per tile (format in paper_2605_18515_amd/csrc/cb_stream.h).  These tests
decode the records independently of the kernel and check that they (1) respect
the batch limits the kernel relies on (16 tiles, 4 payload chunks, 4 panels),
(2) cover every work range's tiles once and in order, (3) point at the codes
and values the tile arrays locate, and (4) multiplied out entry by entry on the
CPU, give exactly the oracle's product on dyadic inputs, where every partial
sum is exact in FP64 whatever the order."""
import numpy as np
import pytest

import oracle
from oracle import cb_model as cm
from paper_2605_18515_amd import matgen

cb = pytest.importorskip("paper_2605_18515_amd.cbspmv", reason="libcbspmv.so not built")

CHUNK, RING, TILES, PANELS = 1024, 4, 16, 4
RINGB = CHUNK * RING
VSIZE = {"f64": 8, "f32": 4, "bf16": 2}


def region(fmt, nz, vtype, blk=16):
    b = cm.tile_region_bytes(int(fmt), int(nz), vtype, blk)
    return (b + 15) // 16 * 16


def value_at(payload, off, vtype):
    if vtype == "f64":
        return float(np.frombuffer(payload[off:off + 8].tobytes(), np.float64)[0])
    if vtype == "f32":
        return float(np.frombuffer(payload[off:off + 4].tobytes(), np.float32)[0])
    bits = np.frombuffer(payload[off:off + 2].tobytes(), np.uint16)[0]
    return float(np.array([np.uint32(bits) << np.uint32(16)], np.uint32).view(np.float32)[0])


def decode(s, info, vtype):
    """Yield (wave, t0, t1, batches) with batches = [(header, records)]."""
    bs = s["batch_stream"].reshape(-1, 4)
    bp, wp = s["batch_ptr"], s["wave_ptr"]
    for w in range(info["nwaves"]):
        o, oe = int(bp[w]), int(bp[w + 1])
        out = []
        while o < oe:
            h = bs[o]
            nt = int(h[2]) & 0xFF
            out.append((h, bs[o + 1:o + 1 + nt]))
            o += 1 + nt
        assert o == oe
        yield w, int(wp[w]), int(wp[w + 1]), out


def check_stream(A, X, vtype="f64", **opts):
    opts.setdefault("spmv_kernel", 0)  # the streaming kernel's batch format
    M = cb.CbMatrix.from_csr(A, device=False, value_type=vtype, **opts)
    info, s = M.info, M.structure()
    M.close()
    vs = VSIZE[vtype]
    S = info["tile_dim"]  # tile size
    assert S == opts.get("tile_dim", 16)
    assert info["stream_bytes"] == 16 * (info["ntiles"] + info["nbatches"])
    assert s["tile_cols"].size == (S * info["ntiles"] if info["col_agg"] else 0)
    assert s["batch_stream"].size == info["stream_bytes"] // 4
    bp = s["batch_ptr"]
    assert bp[0] == 0 and bp[-1] == info["ntiles"] + info["nbatches"] and np.all(np.diff(bp) >= 0)
    row, col, nnz, vp, ty = (s[k].astype(np.int64) for k in ("tile_row", "tile_col", "tile_nnz", "tile_vp",
                                                              "tile_type"))
    agg = bool(info["col_agg"])
    pay = s["payload"]
    y = np.zeros(A.m)
    done_count = np.zeros(max(info["npanels"], 1), np.int64)
    nb = 0
    for w, t0, t1, batches in decode(s, info, vtype):
        if t0 == t1:
            assert not batches
            continue
        B0 = int(vp[t0])
        t = t0
        last_done = {}
        for bi, (h, recs) in enumerate(batches):
            nb += 1
            re_, pb, hz, etot = int(h[0]), int(h[1]), int(h[2]) & 0xFFFFFFFF, int(h[3])
            nt, nflat, ndense, done = hz & 0xFF, (hz >> 8) & 0xFF, (hz >> 16) & 0xFF, hz >> 24
            tiles = list(range(t, t + nt))
            t += nt
            # limits the kernel relies on
            assert 1 <= nt <= TILES and nflat + ndense == nt
            assert row[tiles[0]] == pb and all(0 <= row[i] - pb < PANELS for i in tiles)
            rs = int(vp[tiles[0]]) - B0
            assert re_ == int(vp[tiles[-1]]) - B0 + region(ty[tiles[-1]], nnz[tiles[-1]], vtype, S)
            assert (re_ - 1) // CHUNK - rs // CHUNK + 1 <= RING
            # records: flat tiles in order, then dense tiles in order
            flat = [i for i in tiles if ty[i] != cm.DENSE]
            dense = [i for i in tiles if ty[i] == cm.DENSE]
            assert (len(flat), len(dense)) == (nflat, ndense)
            assert etot == int(sum(nnz[i] for i in flat))
            es = 0
            for r, i in zip(recs, flat + dense):
                rel = int(vp[i]) - B0
                pk = int(r[0]) & 0xFFFFFFFF
                slot, ti = (pk >> 24) & 7, pk >> 27
                assert slot == row[i] % PANELS and ti == i - tiles[0]
                xo = int(r[3])
                assert xo == (s["cols_offset"][row[i]] + S * col[i] if agg else col[i])
                if ty[i] == cm.DENSE:
                    assert pk & 0xFFFFFF == 0 and int(r[1]) == 0 and int(r[2]) == rel
                    continue
                hb = S if ty[i] == cm.CSR else 0
                nz = int(nnz[i])
                assert int(r[2]) == 0
                # positions are kept modulo the 4 KB ring the kernel addresses
                assert (pk & 0xFFF) == (rel + hb - es) % RINGB
                assert ((pk >> 12) & 0xFFF) == (rel + hb + nz + cm.padding(hb + nz, vs) - vs * es) % RINGB
                assert int(r[1]) == es + nz - 1
                es += nz
            # the entries the records point at, multiplied out (through the ring positions, as the
            # kernel addresses them: the batch's bytes lie within four consecutive 1 KB chunks)
            es = 0
            ws = rs // CHUNK * CHUNK  # first byte of the batch's chunk window, relative to B0

            def at(pos):  # payload byte held at ring position pos while this batch is multiplied
                return B0 + ws + (pos % RINGB - ws) % RINGB
            for r, i in zip(recs, flat + dense):
                pk = int(r[0]) & 0xFFFFFFFF
                panel = pb + (((pk >> 24) & 7) - pb) % PANELS
                assert panel == row[i]
                xo = int(r[3])
                if agg:
                    # the tile's S columns the kernel gathers x through, stored (c % 4) * (S / 4) + c // 4
                    tc = s["tile_cols"][S * i:S * i + S].reshape(4, S // 4).T.ravel()
                    width = min(S, s["cols_offset"][row[i] + 1] - xo)
                    assert np.array_equal(tc[:width], s["restore_cols"][xo:xo + width])
                    assert np.all(tc[width:] == s["restore_cols"][s["cols_offset"][row[i]]])
                    orig = lambda c: tc[c]
                else:
                    orig = lambda c: S * xo + c
                if ty[i] == cm.DENSE:
                    base = B0 + int(r[2])
                    for e in range(S * S):
                        if (pay[base + S * S * vs + (e >> 3)] >> (e & 7)) & 1:
                            y[S * panel + e // S] += value_at(pay, base + e * vs, vtype) * X[orig(e % S)]
                    continue
                end = int(r[1])
                for E in range(es, end + 1):
                    code = int(pay[at((pk & 0xFFF) + E)])
                    assert (code & 15) < S and (code >> 4) < S
                    v = value_at(pay, at(((pk >> 12) & 0xFFF) + vs * E), vtype)
                    y[S * panel + (code & 15)] += v * X[orig(code >> 4)]
                es = end + 1
            # done panels: every panel of the range once, in the batch holding its last tile
            for k in range(PANELS):
                if (done >> k) & 1:
                    p = pb + k
                    assert p in set(row[tiles].tolist())
                    assert p not in last_done
                    last_done[p] = bi
                    done_count[p] += 1
        assert t == t1
        panels = sorted(set(row[t0:t1].tolist()))
        assert sorted(last_done) == panels
        for p in panels:
            last_tile = max(i for i in range(t0, t1) if row[i] == p)
            bi = last_done[p]
            first = t0 + sum(int(batches[j][0][2]) & 0xFF for j in range(bi))
            assert first <= last_tile < first + (int(batches[bi][0][2]) & 0xFF)
    assert nb == info["nbatches"]
    return y


def dyadic_case(A, seed=7):
    """Values and x on a dyadic grid (exact in BF16) so every product and partial sum is exact."""
    rng = np.random.default_rng(seed)
    A = matgen.Csr(A.m, A.n, A.row_ptr, A.col_idx, rng.integers(-8, 9, A.nnz).astype(np.float64) / 8)
    return A, rng.integers(-8, 9, A.n).astype(np.float64) / 8


MATS = {
    "lap64": lambda: matgen.laplacian_2d(64),
    "block4": lambda: matgen.block_3d(4, seed=3),
    "poisson8": lambda: matgen.poisson_3d(8),
    "power": lambda: matgen.power_law(3000, seed=5, max_len=2000, window=200),
    "rect": lambda: matgen.random_csr(77, 203, 0.08, 4),
    "dense_mix": lambda: matgen.from_dense(
        np.where(np.random.default_rng(1).random((70, 90)) < np.repeat([0.95, 0.4, 0.05], [32, 20, 18])[:, None],
                 np.random.default_rng(2).uniform(-1, 1, (70, 90)), 0.0)),
    "wide_dense": lambda: matgen.from_dense(np.random.default_rng(4).uniform(-1, 1, (40, 600))),
}


@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("col_agg", [0, 1])
@pytest.mark.parametrize("name", sorted(MATS))
def test_batches_decode_to_the_product(name, col_agg, vtype):
    A, X = dyadic_case(MATS[name]())
    y = check_stream(A, X, vtype, col_agg=col_agg)
    ref = oracle.spmv(A, X)
    assert np.array_equal(y, ref)


@pytest.mark.parametrize("vtype", ["f64", "bf16"])
@pytest.mark.parametrize("col_agg", [0, 1])
@pytest.mark.parametrize("name", sorted(MATS))
def test_batches_decode_to_the_product_8x8(name, col_agg, vtype):
    """8 x 8 tiles (th2 = 40 so that Dense tiles appear where rows are full)."""
    A, X = dyadic_case(MATS[name]())
    y = check_stream(A, X, vtype, col_agg=col_agg, tile_dim=8, th1=8, th2=40)
    assert np.array_equal(y, oracle.spmv(A, X))


@pytest.mark.parametrize("wave_nnz", [64, 300, 5000])
@pytest.mark.parametrize("lb", ["contiguous", "none"])
def test_batches_follow_the_work_ranges(wave_nnz, lb):
    A, X = dyadic_case(matgen.power_law(4000, seed=8, max_len=3000, window=300))
    y = check_stream(A, X, "f64", lb_mode=lb, wave_nnz=wave_nnz, quantum_tiles=3)
    assert np.array_equal(y, oracle.spmv(A, X))


def test_paper_mode_has_no_records():
    A = matgen.laplacian_2d(20)
    M = cb.CbMatrix.from_csr(A, device=False, lb_mode="paper")
    info, s = M.info, M.structure()
    M.close()
    assert info["nbatches"] == 0 and info["stream_bytes"] == 0
    assert s["batch_stream"].size == 0 and s["batch_ptr"].size == 0 and s["tile_cols"].size == 0


def test_limits_cut_batches():
    # a single 16-row panel of 40 dense-ish tiles: the 16-tile limit and the 4-chunk limit both cut
    A, X = dyadic_case(matgen.from_dense(np.random.default_rng(3).uniform(-1, 1, (16, 640))))
    M = cb.CbMatrix.from_csr(A, device=False, col_agg=0, spmv_kernel=0)
    info = M.info
    M.close()
    assert info["tiles_dense"] == 40
    # a Dense FP64 region is 2080 bytes, so a batch holds at most two of them
    assert info["nbatches"] >= 20
    assert np.array_equal(check_stream(A, X, "f64", col_agg=0), oracle.spmv(A, X))
    # one tile per panel over many panels: the 4-panel limit cuts
    A2, X2 = dyadic_case(matgen.identity(16 * 40))
    M = cb.CbMatrix.from_csr(A2, device=False, spmv_kernel=0)
    info2 = M.info
    M.close()
    assert info2["nbatches"] >= 5
    assert np.array_equal(check_stream(A2, X2, "f64"), oracle.spmv(A2, X2))
