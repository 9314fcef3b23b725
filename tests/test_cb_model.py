"""Pins of the conversion oracle (oracle/cb_model.py): a hand-worked example,
brute force on dense patterns, threshold edges, an independent re-statement of
Algorithm 2's greedy choice, and the paper's storage model."""
import json
import os
import struct

import numpy as np
import pytest

import oracle
from oracle import cb_model as cm
from paper_2605_18515_amd import matgen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    return json.load(open(os.path.join(GOLD, name)))


def worked_csr():
    g = golden("cb_worked_example.json")
    D = np.zeros((g["m"], g["n"]))
    for r, c, v in g["entries"]:
        D[r, c] = v
    return g, matgen.from_dense(D)


def test_paper_constants():
    c = golden("paper_constants.json")
    assert cm.BLK == c["block_size"]["value"]
    assert cm.SUPER_SPARSE == c["super_sparse_below"]["value"]
    assert cm.TH0 == c["th0"]["value"] and cm.TH1 == c["th1"]["value"] and cm.TH2 == c["th2"]["value"]
    assert cm.WARPS_PER_TB == c["warps_per_thread_block"]["value"]
    assert cm.bytes_model_cb(1, 0) == c["cb_storage_bytes_per_block"]["value"]
    assert cm.bytes_model_cb(0, 1) == c["cb_storage_bytes_per_nnz"]["value"]


def test_worked_example_plain_partition():
    g, A = worked_csr()
    tiles = cm.plain_tiles(A.row_ptr, A.col_idx)
    got = sorted([p, c, len(e)] for (p, c), e in tiles.items())
    assert got == g["plain"]["tiles"]
    assert cm.super_sparse_share(tiles) == g["plain"]["share"]


def _check_tiles(model, exp_tiles, vtype, A):
    vps, _ = cm.layout(model, vtype)
    buf = cm.pack(model, A.values, vtype, rounder=oracle.round_f32_bits)
    assert len(model.tiles) == len(exp_tiles)
    for t, vp, e in zip(model.tiles, vps, exp_tiles):
        assert (t.panel, t.tcol, t.fmt, t.nnz, vp) == (e["panel"], e["tcol"], e["fmt"], e["nnz"], e["vp"])
        assert list(buf[vp:vp + t.nnz]) == e["codes"]
        vo = e["value_offset"]
        vals = struct.unpack_from("<%dd" % t.nnz, buf, vp + vo)
        assert list(vals) == e["values"]
        dec = cm.decode_tile(buf, vp, t.fmt, t.nnz, vtype)
        assert [cm.pack_code(lr, lc) for lr, lc, _ in dec] == e["codes"]


def test_worked_example_aggregated():
    g, A = worked_csr()
    ex = g["aggregated_f64"]
    model = cm.build(A.m, A.n, A.row_ptr, A.col_idx)
    assert model.col_agg
    assert model.restore_cols.tolist() == ex["restore_cols"]
    assert model.cols_offset.tolist() == ex["cols_offset"]
    _check_tiles(model, ex["tiles"], "f64", A)
    assert cm.layout(model, "f64")[1] == ex["payload_bytes"]
    end, order, T = cm.lb_paper([t.nnz for t in model.tiles])
    assert end == ex["lb_end"]
    f32 = g["aggregated_f32"]
    vps, total = cm.layout(model, "f32")
    assert vps == f32["vps"] and total == f32["payload_bytes"]
    for t, vo in zip(model.tiles, f32["value_offsets"]):
        assert t.nnz + cm.padding(t.nnz, 4) == vo


def test_worked_example_plain():
    g, A = worked_csr()
    ex = g["plain_f64"]
    model = cm.build(A.m, A.n, A.row_ptr, A.col_idx, col_agg_mode=0)
    assert not model.col_agg
    _check_tiles(model, ex["tiles"], "f64", A)
    assert cm.layout(model, "f64")[1] == ex["payload_bytes"]
    assert cm.lb_paper([t.nnz for t in model.tiles])[0] == ex["lb_end"]
    assert cm.bytes_model_cb(len(model.tiles), A.nnz) == ex["bytes_model_cb"]


def test_worked_example_csr_and_dense():
    g, A = worked_csr()
    ex = g["plain_th1_2_th2_2_f64"]
    model = cm.build(A.m, A.n, A.row_ptr, A.col_idx, col_agg_mode=0, th1=ex["th1"], th2=ex["th2"])
    assert [t.fmt for t in model.tiles] == ex["fmts"]
    vps, total = cm.layout(model, "f64")
    assert vps == ex["vps"] and total == ex["payload_bytes"]
    buf = cm.pack(model, A.values, "f64")
    dense = struct.unpack_from("<256d", buf, 0)
    for slot, v in enumerate(dense):
        assert v == ex["dense_nonzero_value_slots"].get(str(slot), 0.0)
    mask = buf[2048:2080]
    for b in range(32):
        assert mask[b] == ex["dense_mask_bytes"].get(str(b), 0)
    vp = vps[1]
    assert list(buf[vp:vp + 16]) == ex["csr_row_starts"]
    assert list(buf[vp + 16:vp + 18]) == ex["csr_codes"]
    assert struct.unpack_from("<2d", buf, vp + ex["csr_value_offset"]) == (2.0, 6.0)
    # every tile decodes back to its entries
    for t, vpt in zip(model.tiles, vps):
        dec = cm.decode_tile(buf, vpt, t.fmt, t.nnz, "f64")
        assert [(lr, lc) for lr, lc, _ in dec] == [(lr, lc) for lr, lc, _ in t.entries]


def _dense_pattern(A):
    P = np.zeros((A.m, A.n), dtype=bool)
    P[A.rows(), A.col_idx] = True
    return P


@pytest.mark.parametrize("blk", [8, 16])
@pytest.mark.parametrize("seed", range(5))
def test_plain_partition_brute_force(seed, blk):
    rng = np.random.default_rng(seed)
    m, n = int(rng.integers(1, 70)), int(rng.integers(1, 70))
    A = matgen.random_csr(m, n, float(rng.uniform(0.02, 0.5)), seed)
    P = _dense_pattern(A)
    tiles = cm.plain_tiles(A.row_ptr, A.col_idx, blk)
    expect = {}
    for p in range(0, m, blk):
        for c in range(0, n, blk):
            cnt = int(P[p:p + blk, c:c + blk].sum())
            if cnt:
                expect[(p // blk, c // blk)] = cnt
    assert {k: len(v) for k, v in tiles.items()} == expect
    for (p, c), ent in tiles.items():
        for lr, lc, t in ent:
            assert A.rows()[t] == blk * p + lr and A.col_idx[t] == blk * c + lc


@pytest.mark.parametrize("blk", [8, 16])
@pytest.mark.parametrize("seed", range(5))
def test_column_aggregation_brute_force(seed, blk):
    rng = np.random.default_rng(50 + seed)
    m, n = int(rng.integers(1, 60)), int(rng.integers(1, 300))
    A = matgen.random_csr(m, n, float(rng.uniform(0.01, 0.2)), seed)
    P = _dense_pattern(A)
    restore, offs, tiles = cm.aggregate_columns(m, A.row_ptr, A.col_idx, blk)
    got = {k: len(v) for k, v in tiles.items()}
    expect, rc = {}, []
    for p in range(0, m, blk):
        sub = P[p:p + blk]
        keep = np.nonzero(sub.any(axis=0))[0]       # non-empty columns, shifted left
        rc.extend(keep.tolist())
        packed = sub[:, keep]
        for c in range(0, packed.shape[1], blk):
            expect[(p // blk, c // blk)] = int(packed[:, c:c + blk].sum())
    assert got == expect
    assert restore.tolist() == rc
    # every chunk but a panel's last holds exactly blk non-empty columns, so >= blk entries
    for p in range((m + blk - 1) // blk):
        ncols = int(offs[p + 1] - offs[p])
        for c in range((ncols + blk - 1) // blk):
            if c < (ncols + blk - 1) // blk - 1:
                assert got[(p, c)] >= blk
    # original coordinates come back through restore_cols / cols_offset
    for (p, c), ent in tiles.items():
        for lr, lc, t in ent:
            assert restore[offs[p] + blk * c + lc] == A.col_idx[t]
            assert A.rows()[t] == blk * p + lr


def test_format_threshold_edges():
    assert [cm.select_format(v) for v in (0, 1, 31, 32, 33, 127, 128, 129, 256)] == \
        [cm.COO, cm.COO, cm.COO, cm.CSR, cm.CSR, cm.CSR, cm.CSR, cm.DENSE, cm.DENSE]


def test_th0_decision_edges():
    assert cm.decide_col_agg(0.15) and cm.decide_col_agg(0.9)
    assert not cm.decide_col_agg(0.1499999)
    assert not cm.decide_col_agg(0.9, mode=0) and cm.decide_col_agg(0.0, mode=1)
    # a matrix whose every tile is full (256 entries) has share 0: no aggregation
    D = np.ones((32, 32))
    A = matgen.from_dense(D)
    mdl = cm.build(32, 32, A.row_ptr, A.col_idx)
    assert mdl.share == 0.0 and not mdl.col_agg and all(t.fmt == cm.DENSE for t in mdl.tiles)
    # share exactly 3/20 = 0.15 -> applied; 2/20 -> not
    def mat(n_sparse, n_dense=17):
        blocks = []
        for b in range(n_sparse + n_dense):
            B = np.zeros((16, 16))
            if b < n_sparse:
                B[0, 0] = 1.0
            else:
                B[:, :] = 1.0
            blocks.append(B)
        return matgen.from_dense(np.hstack(blocks))
    A3 = mat(3)
    assert abs(cm.build(A3.m, A3.n, A3.row_ptr, A3.col_idx).share - 0.15) < 1e-15
    assert cm.build(A3.m, A3.n, A3.row_ptr, A3.col_idx).col_agg
    A2 = mat(2, 18)
    assert not cm.build(A2.m, A2.n, A2.row_ptr, A2.col_idx).col_agg


def test_lb_worked_example():
    g = golden("lb_worked_example.json")
    end, order, T = cm.lb_paper(g["nnz"], g["W"])
    assert T == g["T"] and end == g["end"] and order == g["order"]
    assert cm.lb_quantum_loads(g["nnz"], end, T, g["W"]).tolist() == g["tb_loads"]


def _lpt_scan(nnz, W):
    """Independent statement of the greedy choice: each block, taken in
    descending nnz order, goes to the least-loaded thread block that still has
    room (smallest id on ties), into its next free slot."""
    T = (len(nnz) + W - 1) // W
    loads, fill = [0] * T, [0] * T
    end = [0] * len(nnz)
    for i in sorted(range(len(nnz)), key=lambda i: (-nnz[i], i)):
        best = min((tb for tb in range(T) if fill[tb] < W), key=lambda tb: (loads[tb], tb))
        end[i] = best * W + fill[best]
        loads[best] += nnz[i]
        fill[best] += 1
    return end


@pytest.mark.parametrize("seed", range(8))
def test_lb_matches_independent_scan(seed):
    rng = np.random.default_rng(seed)
    nb = int(rng.integers(1, 300))
    W = int(rng.choice([1, 2, 3, 8]))
    nnz = rng.integers(0, 257, nb).tolist()
    end, order, T = cm.lb_paper(nnz, W)
    assert end == _lpt_scan(nnz, W)
    assert len(set(end)) == nb and all(0 <= e < T * W for e in end)
    assert sorted(order) == list(range(nb))
    assert [end[i] for i in order] == sorted(end)


def test_lb_balances_better_than_round_robin():
    rng = np.random.default_rng(3)
    nnz = np.minimum(rng.zipf(1.8, 4000), 256).tolist()
    end, _, T = cm.lb_paper(nnz, 8)
    lpt = cm.lb_quantum_loads(nnz, end, T)
    naive = cm.lb_quantum_loads(nnz, list(range(len(nnz))), T)
    assert lpt.std() < naive.std() and lpt.max() <= naive.max()


def test_storage_model_all_coo():
    """Section 4.4.1: with every tile COO and no aggregation, the packed values
    and codes take 9 bytes per entry plus padding; the high-level arrays take
    4+4+4+1+8 bytes per tile."""
    A = matgen.random_csr(150, 170, 0.05, 12)
    model = cm.build(A.m, A.n, A.row_ptr, A.col_idx, col_agg_mode=0, th1=10 ** 6, th2=10 ** 6)
    assert all(t.fmt == cm.COO for t in model.tiles)
    raw = sum(cm.tile_region_bytes(cm.COO, t.nnz, "f64") for t in model.tiles)
    pads = sum(cm.padding(t.nnz, 8) for t in model.tiles)
    assert raw == 9 * A.nnz + pads
    assert cm.bytes_model_cb(len(model.tiles), A.nnz) == 21 * len(model.tiles) + 9 * A.nnz
    assert cm.bytes_model_csr(A.m, A.nnz) == (A.m + 1) * 4 + 12 * A.nnz
    assert cm.bytes_model_bsr(len(model.tiles), 10) == 2048 * len(model.tiles) + 44 + 4 * len(model.tiles)


def test_padding_formula():
    # Algorithm 3: (nnz * size(Idx)) mod size(Val), complemented when non-zero
    assert [cm.padding(k, 8) for k in range(10)] == [0, 7, 6, 5, 4, 3, 2, 1, 0, 7]
    assert [cm.padding(k, 4) for k in range(6)] == [0, 3, 2, 1, 0, 3]
    assert [cm.padding(k, 2) for k in range(4)] == [0, 1, 0, 1]


def test_code_nibbles():
    # Algorithm 3: row = b & 15, col = b >> 4
    for lr in range(16):
        for lc in range(16):
            b = cm.pack_code(lr, lc)
            assert 0 <= b < 256 and (b & 15, b >> 4) == (lr, lc)


@pytest.mark.parametrize("blk", [8, 16])
@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
def test_pack_decode_round_trip(vtype, blk):
    rng = np.random.default_rng(21)
    dens = np.repeat([0.9, 0.35, 0.04], [32, 32, 26])[:, None]
    D = np.where(rng.random((90, 75)) < dens, rng.uniform(-1, 1, (90, 75)), 0.0)
    A = matgen.from_dense(D)
    rounder = {"f32": oracle.round_f32_bits, "bf16": oracle.round_bf16_bits, "f64": None}[vtype]
    th1, th2 = (20, 60) if blk == 16 else (6, 40)
    for agg in (0, 1):
        model = cm.build(A.m, A.n, A.row_ptr, A.col_idx, col_agg_mode=agg, th1=th1, th2=th2, blk=blk)
        assert {t.fmt for t in model.tiles} == {cm.COO, cm.CSR, cm.DENSE}
        buf = cm.pack(model, A.values, vtype, rounder)
        vps, _ = cm.layout(model, vtype)
        bits = cm.value_bits(A.values, vtype, rounder)
        for t, vp in zip(model.tiles, vps):
            assert vp % cm.TILE_ALIGN == 0
            dec = cm.decode_tile(buf, vp, t.fmt, t.nnz, vtype, blk)
            assert [(lr, lc, int(bits[i])) for lr, lc, i in t.entries] == [(a, b, int(c)) for a, b, c in dec]


def _check_worked8(ex, model, A):
    buf = cm.pack(model, A.values, "f64")
    vps, total = cm.layout(model, "f64")
    assert total == ex["payload_bytes"] == len(buf)
    assert [(t.panel, t.tcol, t.fmt, t.nnz, vp) for t, vp in zip(model.tiles, vps)] == \
        [(e["panel"], e["tcol"], e["fmt"], e["nnz"], e["vp"]) for e in ex["tiles"]]
    dense = struct.unpack_from("<64d", buf, 0)
    for slot, v in enumerate(dense):
        assert v == ex["dense_value_slots"].get(str(slot), 0.0)
    assert list(buf[512:520]) == ex["dense_mask"]
    vp = ex["tiles"][1]["vp"]
    nc = len(ex["csr_codes"])
    assert list(buf[vp:vp + 8]) == ex["csr_row_starts"]
    assert list(buf[vp + 8:vp + 8 + nc]) == ex["csr_codes"]
    assert list(struct.unpack_from("<%dd" % nc, buf, vp + ex["csr_value_offset"])) == ex["csr_values"]
    for t, vpt in zip(model.tiles, vps):
        dec = cm.decode_tile(buf, vpt, t.fmt, t.nnz, "f64", 8)
        assert [(lr, lc) for lr, lc, _ in dec] == [(lr, lc) for lr, lc, _ in t.entries]
    return buf, vps


def test_worked_example_8x8():
    """Sub-block size 8: a hand-worked conversion (tests/golden/cb8_worked_example.json)."""
    g = golden("cb8_worked_example.json")
    D = np.zeros((g["m"], g["n"]))
    for r, c, v in g["entries"]:
        D[r, c] = v
    A = matgen.from_dense(D)
    assert cm.super_sparse_share(cm.plain_tiles(A.row_ptr, A.col_idx)) == g["share_16"]["share"]
    ex = g["plain_f64"]
    model = cm.build(A.m, A.n, A.row_ptr, A.col_idx, col_agg_mode=0, th1=g["th1"], th2=g["th2"], blk=8)
    assert not model.col_agg and model.blk == 8
    buf, vps = _check_worked8(ex, model, A)
    for t, vp, e in zip(model.tiles[2:], vps[2:], ex["coo"]):
        assert list(buf[vp:vp + t.nnz]) == e["codes"]
        assert list(struct.unpack_from("<%dd" % t.nnz, buf, vp + e["value_offset"])) == e["values"]
    ex = g["aggregated_f64"]
    model = cm.build(A.m, A.n, A.row_ptr, A.col_idx, th1=g["th1"], th2=g["th2"], blk=8)
    assert model.col_agg
    assert model.restore_cols.tolist() == ex["restore_cols"]
    assert model.cols_offset.tolist() == ex["cols_offset"]
    _check_worked8(ex, model, A)


def test_unknown_sub_block_size_is_refused():
    A = matgen.identity(4)
    with pytest.raises(ValueError):
        cm.build(A.m, A.n, A.row_ptr, A.col_idx, blk=32)
