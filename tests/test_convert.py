"""Host-side checks of the library (no GPU): the C ABI loads and exports every
declared symbol; the C++ converter reproduces the conversion oracle bit for bit
(tiles, formats, aggregation arrays, packed bytes, Algorithm 2 groups); CSR
round trips are exact; malformed input is rejected with a status."""
import ctypes

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from oracle import cb_model as cm
from paper_2605_18515_amd import matgen

cb = pytest.importorskip("paper_2605_18515_amd.cbspmv", reason="libcbspmv.so not built")

VT = {"f64": cb.CB_VALUE_F64, "f32": cb.CB_VALUE_F32, "bf16": cb.CB_VALUE_BF16}
ROUNDER = {"f64": None, "f32": oracle.round_f32_bits, "bf16": oracle.round_bf16_bits}


def test_every_declared_symbol_is_exported():
    names = cb.header_functions()
    assert len(names) >= 11
    lib = cb.library_handle()
    for nm in names:
        assert hasattr(lib, nm), nm
    for required in ("cb_create", "cb_spmv", "cb_spmm", "cb_destroy"):
        assert required in names


def test_struct_sizes_match_header():
    o = cb.cb_options_default()
    assert o.struct_size == ctypes.sizeof(cb.CbOptions)
    assert o.th1 == 32 and o.th2 == 128 and abs(o.th0 - 0.15) == 0 and o.quantum_tiles == 8 and o.col_agg == -1
    A = matgen.identity(5)
    h = cb.cb_create_host(5, 5, 5, A.row_ptr, A.col_idx, A.values)
    assert cb.cb_get_info(h)["struct_size"] == ctypes.sizeof(cb.CbInfo)
    cb.cb_destroy(h)


def host_matrix(A, **opts):
    return cb.CbMatrix.from_csr(A, device=False, **opts)


def check_against_model(A, vtype="f64", col_agg=-1, th1=32, th2=128, lb="contiguous", W=8, th0=0.15, tile_dim=16):
    M = host_matrix(A, value_type=vtype, col_agg=col_agg, th1=th1, th2=th2, lb_mode=lb, quantum_tiles=W, th0=th0,
                    tile_dim=tile_dim)
    info, s = M.info, M.structure()
    assert info["tile_dim"] == tile_dim
    model = cm.build(A.m, A.n, A.row_ptr, A.col_idx, col_agg_mode=col_agg, th0=th0, th1=th1, th2=th2, blk=tile_dim)
    NT = len(model.tiles)
    assert info["ntiles"] == NT
    assert info["col_agg"] == int(model.col_agg)
    assert info["super_sparse_share"] == model.share
    assert [info["tiles_coo"], info["tiles_csr"], info["tiles_dense"]] == \
        [sum(t.fmt == f for t in model.tiles) for f in (cm.COO, cm.CSR, cm.DENSE)]
    assert info["meta_bytes"] == 21 * NT
    # natural order view of the kernel-order arrays
    ori = s["tile_ori"]
    assert sorted(ori.tolist()) == list(range(NT))
    nat = np.empty(NT, np.int64)
    nat[ori] = np.arange(NT)
    vps, total = cm.layout(model, vtype)
    assert info["payload_bytes"] == total
    for i, t in enumerate(model.tiles):
        j = nat[i]
        assert (s["tile_row"][j], s["tile_col"][j], s["tile_nnz"][j], s["tile_type"][j], s["tile_vp"][j]) == \
            (t.panel, t.tcol, t.nnz, t.fmt, vps[i]), i
    assert bytes(s["payload"]) == cm.pack(model, A.values, vtype, ROUNDER[vtype])
    if model.col_agg:
        assert np.array_equal(s["restore_cols"], model.restore_cols)
        assert np.array_equal(s["cols_offset"], model.cols_offset)
        assert np.array_equal(s["tile_xoff"], s["cols_offset"][s["tile_row"]] + tile_dim * s["tile_col"])
    else:
        assert s["tile_xoff"].size == 0
    # grouping
    if lb == "paper":
        end, order, T = cm.lb_paper([t.nnz for t in model.tiles], W)
        assert ori.tolist() == order
        qp = s["quantum_ptr"]
        assert len(qp) == T + 1 and qp[0] == 0 and qp[-1] == NT
        for b in range(T):
            assert all(end[ori[k]] // W == b for k in range(qp[b], qp[b + 1]))
    elif lb == "none":
        assert ori.tolist() == list(range(NT))
        assert s["quantum_ptr"].tolist() == [min(NT, b * W) for b in range((NT + W - 1) // W + 1)]
    else:
        assert ori.tolist() == list(range(NT))
    wp = s["wave_ptr"]
    assert wp[0] == 0 and wp[-1] == NT and (NT == 0 or np.all(np.diff(wp) > 0))
    # panel ownership: one run inside one work range
    runs = np.zeros(info["npanels"], int)
    for w in range(len(wp) - 1):
        for k in range(wp[w], wp[w + 1]):
            if k == wp[w] or s["tile_row"][k] != s["tile_row"][k - 1]:
                runs[s["tile_row"][k]] += 1
    assert np.array_equal(s["panel_shared"], (runs > 1).astype(np.uint8))
    assert s["prepass_list"].tolist() == np.nonzero(runs != 1)[0].tolist()
    M.close()
    return info, s, model


MATS = {
    "lap64": lambda: matgen.laplacian_2d(64),
    "lap13": lambda: matgen.laplacian_2d(13),
    "block4": lambda: matgen.block_3d(4, seed=3),
    "poisson6": lambda: matgen.poisson_3d(6),
    "power": lambda: matgen.power_law(3000, seed=5, max_len=2000, window=200),
    "rect": lambda: matgen.random_csr(77, 203, 0.08, 4),
    "dense_mix": lambda: matgen.from_dense(
        np.where(np.random.default_rng(1).random((70, 90)) < np.repeat([0.95, 0.4, 0.05], [32, 20, 18])[:, None],
                 np.random.default_rng(2).uniform(-1, 1, (70, 90)), 0.0)),
}


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("col_agg", [-1, 0, 1])
def test_converter_matches_model(name, col_agg):
    check_against_model(MATS[name](), col_agg=col_agg)


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("col_agg", [-1, 0, 1])
def test_converter_matches_model_8x8(name, col_agg):
    check_against_model(MATS[name](), col_agg=col_agg, tile_dim=8, th1=8, th2=40)


@pytest.mark.parametrize("lb", ["paper", "none"])
@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
def test_converter_matches_model_8x8_every_mode(vtype, lb):
    info, _, _ = check_against_model(MATS["dense_mix"](), vtype=vtype, col_agg=0, tile_dim=8, th1=8, th2=40, lb=lb,
                                     W=3)
    assert info["tiles_coo"] and info["tiles_csr"] and info["tiles_dense"]


def test_tile_dim_is_checked():
    A = matgen.laplacian_2d(8)
    for bad in (4, 32, -1, 17):
        with pytest.raises(cb.CbError) as e:
            host_matrix(A, tile_dim=bad)
        assert e.value.status == cb.CB_ERROR_INVALID_VALUE
    with pytest.raises(cb.CbError) as e:
        host_matrix(A, tile_dim=8, spmv_kernel=1)
    assert e.value.status == cb.CB_ERROR_NOT_SUPPORTED
    M = host_matrix(A, tile_dim=0)
    assert M.info["tile_dim"] == 16
    M.close()


@pytest.mark.parametrize("vtype", ["f32", "bf16"])
@pytest.mark.parametrize("name", ["dense_mix", "power"])
def test_converter_matches_model_low_precision(vtype, name):
    check_against_model(MATS[name](), vtype=vtype, col_agg=1, th1=20, th2=60)


@pytest.mark.parametrize("lb", ["paper", "none"])
@pytest.mark.parametrize("W", [1, 3, 8])
@pytest.mark.parametrize("name", ["dense_mix", "power", "lap13"])
def test_grouping_modes_match_model(name, lb, W):
    check_against_model(MATS[name](), lb=lb, W=W)


def test_thresholds_reach_every_format():
    info, _, _ = check_against_model(MATS["dense_mix"](), col_agg=0, th1=20, th2=60)
    assert info["tiles_coo"] and info["tiles_csr"] and info["tiles_dense"]


@pytest.mark.parametrize("nz", [0, 1, 2, 15, 16, 31, 32, 33, 64, 127, 128, 129, 200, 255, 256])
def test_single_tile_sweep(nz):
    A = matgen.single_tile(nz, seed=nz)
    info, s, model = check_against_model(A, col_agg=0)
    if nz:
        assert s["tile_type"][0] == cm.select_format(nz)
    rp, ci, va = host_matrix(A).export_csr()
    assert np.array_equal(rp, A.row_ptr) and np.array_equal(ci, A.col_idx)
    assert np.array_equal(va.view(np.uint64), A.values.view(np.uint64))


def roundtrip(A, vtype="f64", **opts):
    M = host_matrix(A, value_type=vtype, **opts)
    rp, ci, va = M.export_csr()
    assert np.array_equal(rp, A.row_ptr)
    assert np.array_equal(ci, A.col_idx)
    if vtype == "f64":
        assert np.array_equal(va.view(np.uint64), A.values.view(np.uint64))
    elif vtype == "f32":
        assert np.array_equal(va.view(np.uint32), oracle.round_f32_bits(A.values))
    else:
        assert np.array_equal(va, oracle.round_bf16_bits(A.values))
    M.close()


@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("name", sorted(MATS))
def test_round_trip(name, vtype):
    for agg in (0, 1):
        for lb in ("contiguous", "paper"):
            roundtrip(MATS[name](), vtype, col_agg=agg, th1=20, th2=60, lb_mode=lb)
            roundtrip(MATS[name](), vtype, col_agg=agg, th1=8, th2=40, lb_mode=lb, tile_dim=8)


def test_round_trip_special_values():
    rng = np.random.default_rng(7)
    D = np.zeros((40, 40))
    keep = rng.random((40, 40)) < 0.6
    D[keep] = rng.choice([0.0, -0.0, np.nan, np.inf, -np.inf, 1e-310, -5e-324, 1.5, 3.4e38, 1e300], keep.sum())
    A = matgen.from_dense(D, keep_zeros_mask=keep)
    assert A.nnz == keep.sum()
    for vt in ("f64", "f32", "bf16"):
        for th2 in (128, 5):  # th2 = 5 forces Dense tiles, whose zero fill must not swallow stored zeros
            for td in (16, 8):
                roundtrip(A, vt, col_agg=0, th1=2, th2=th2, tile_dim=td)
                roundtrip(A, vt, col_agg=1, th1=2, th2=th2, tile_dim=td)


def test_empty_shapes():
    for m, n in [(0, 0), (0, 7), (7, 0), (33, 17)]:
        A = matgen.Csr(m, n, np.zeros(m + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
        M = host_matrix(A)
        inf = M.info
        assert inf["ntiles"] == 0 and inf["npanels"] == (m + 15) // 16
        assert inf["prepass_panels"] == inf["npanels"]  # every (empty) panel is written by the pre-pass
        rp, ci, va = M.export_csr()
        assert np.array_equal(rp, A.row_ptr) and ci.size == 0
        M.close()


def test_empty_rows_and_panels():
    D = np.zeros((100, 60))
    D[3, 5] = 1.0
    D[70, 59] = 2.0
    D[99, 0] = 3.0
    A = matgen.from_dense(D)
    info, s, _ = check_against_model(A)
    assert set(s["prepass_list"].tolist()) == {1, 2, 3, 5}
    roundtrip(A)


def test_wide_rows_split_contiguous():
    # one row with 5000 entries: its panel is heavier than twice the range target and is split
    A = matgen.power_law(600, seed=9, max_len=600, window=100)
    rp = np.array([0, 5000] + [5000] * 15, np.int64)
    B = matgen.Csr(16, 6000, rp, np.arange(0, 6000, 6000 / 5000).astype(np.int32)[:5000], np.ones(5000))
    info, s, _ = check_against_model(B, col_agg=0)
    assert info["nwaves"] > 1 and info["shared_panels"] == 1 and s["prepass_list"].tolist() == [0]
    M = host_matrix(B, col_agg=0, wave_nnz=256)
    assert M.info["nwaves"] >= 5000 // 256
    check_against_model(A)


def test_contiguous_ranges_are_balanced():
    A = matgen.block_3d(8, seed=1)
    M = host_matrix(A, wave_nnz=2000)
    inf, s = M.info, M.structure()
    w = np.array([s["tile_nnz"][s["wave_ptr"][i]:s["wave_ptr"][i + 1]].sum() for i in range(inf["nwaves"])])
    assert w.max() <= 2000 + 8 * 100 and inf["shared_panels"] == 0
    assert inf["wave_nnz_max"] == w.max()


def test_storage_model_matches_paper_widths():
    A = matgen.random_csr(200, 230, 0.03, 8)
    M = host_matrix(A, col_agg=0, th1=1000, th2=1000)
    inf, s = M.info, M.structure()
    assert inf["tiles_coo"] == inf["ntiles"]
    pads = sum(cm.padding(int(z), 8) for z in s["tile_nnz"])
    raw = 9 * A.nnz + pads
    align = sum((-cm.tile_region_bytes(cm.COO, int(z), "f64")) % 16 for z in s["tile_nnz"])
    assert inf["payload_bytes"] == raw + align
    assert inf["meta_bytes"] + 9 * A.nnz == cm.bytes_model_cb(inf["ntiles"], A.nnz)


def _status(fn, *a):
    try:
        fn(*a)
    except cb.CbError as e:
        return e.status, str(e)
    return 0, ""


@pytest.mark.parametrize("case", ["rp0", "rpm", "decreasing", "col_range", "col_neg", "unsorted", "duplicate",
                                  "neg_m", "null_cols", "huge"])
def test_malformed_csr_is_rejected(case):
    rp = np.array([0, 2, 3, 5], np.int64)
    ci = np.array([0, 2, 1, 0, 3], np.int32)
    va = np.ones(5)
    m, n, nnz = 3, 4, 5
    if case == "rp0":
        rp = rp.copy(); rp[0] = 1
    elif case == "rpm":
        nnz = 4
    elif case == "decreasing":
        rp = np.array([0, 3, 2, 5], np.int64)
    elif case == "col_range":
        ci = ci.copy(); ci[4] = 4
    elif case == "col_neg":
        ci = ci.copy(); ci[2] = -1
    elif case == "unsorted":
        ci = np.array([2, 0, 1, 0, 3], np.int32)
    elif case == "duplicate":
        ci = np.array([0, 0, 1, 0, 3], np.int32)
    elif case == "neg_m":
        m = -1
    elif case == "huge":
        n = 1 << 31
    if case == "null_cols":
        h = ctypes.c_void_p()
        st = cb.library_handle().cb_create_host(ctypes.byref(h), 3, 4, 5, rp.ctypes.data, None, va.ctypes.data, None)
        assert st == cb.CB_ERROR_INVALID_VALUE and "NULL" in cb.cb_last_error()
        return
    st, msg = _status(cb.cb_create_host, m, n, nnz, rp, ci, va)
    assert st == cb.CB_ERROR_INVALID_VALUE, (case, st, msg)
    assert msg


def test_bad_options_are_rejected():
    A = matgen.identity(20)
    for k, v in [("value_type", 3), ("col_agg", 2), ("th1", -1), ("quantum_tiles", 0), ("lb_mode", 7),
                 ("wave_nnz", -5), ("th0", float("nan")), ("row_reduce", 5), ("row_reduce", -2),
                 ("vector_f64", 2), ("vector_f64", -1)]:
        o = cb.cb_options_default()
        setattr(o, k, v)
        st, _ = _status(cb.cb_create_host, 20, 20, 20, A.row_ptr, A.col_idx, A.values, o)
        assert st == cb.CB_ERROR_INVALID_VALUE, k
    o = cb.cb_options_default()
    o.struct_size = 12
    assert _status(cb.cb_create_host, 20, 20, 20, A.row_ptr, A.col_idx, A.values, o)[0] == cb.CB_ERROR_INVALID_VALUE


def test_row_reduce_resolution_and_run_statistic():
    # 2 x 2 block diagonal pattern: one 16 x 16 tile, rows 0-15 with 2 entries each in one run
    n = 16
    rows = np.repeat(np.arange(n), 2)
    cols = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
    cols.sort(axis=1)
    A = matgen.Csr(n, n, np.arange(0, 2 * n + 1, 2, dtype=np.int64), cols.ravel().astype(np.int32),
                   np.ones(2 * n))
    assert rows.size == A.nnz
    # runs of two entries per tile row: the two-copy accumulator modes for the streaming kernel; the
    # quad kernel (chosen here automatically: 32 entries in runs) sums a lane's runs itself and keeps
    # one copy
    for vt, want in (("f64", 3), ("f32", 4), ("bf16", 4)):
        M = cb.CbMatrix.from_csr(A, device=False, value_type=vt, th1=64, th2=256, spmv_kernel=0)
        assert M.info["row_reduce"] == want and M.info["flat_run_mean"] == 2.0
        M.close()
    for vt, want in (("f64", 0), ("f32", 2), ("bf16", 2)):
        M = cb.CbMatrix.from_csr(A, device=False, value_type=vt, th1=64, th2=256)
        assert M.info["spmv_kernel"] == 2 and M.info["row_reduce"] == want
        M.close()
    # one entry per tile row (a permutation matrix): one copy
    P = matgen.Csr(n, n, np.arange(n + 1, dtype=np.int64), ((np.arange(n) * 5) % n).astype(np.int32), np.ones(n))
    for vt, want in (("f64", 0), ("f32", 2)):
        M = cb.CbMatrix.from_csr(P, device=False, value_type=vt)
        assert M.info["row_reduce"] == want and M.info["flat_run_mean"] == 1.0
        M.close()
    for rr in (0, 1, 2, 3, 4):
        M = cb.CbMatrix.from_csr(A, device=False, row_reduce=rr, spmv_kernel=0)
        assert M.info["row_reduce"] == rr
        M.close()
    # double vectors: always with FP64 storage, on request with FP32/BF16 (then FP64 atomics suffice)
    for vt, wide, want in (("f64", 0, 1), ("f32", 0, 0), ("f32", 1, 1), ("bf16", 1, 1)):
        M = cb.CbMatrix.from_csr(A, device=False, value_type=vt, vector_f64=wide, spmv_kernel=0)
        assert M.info["vector_f64"] == want
        assert M.info["row_reduce"] == (3 if want else 4)
        M.close()


def test_host_handle_cannot_multiply():
    A = matgen.identity(20)
    h = cb.cb_create_host(20, 20, 20, A.row_ptr, A.col_idx, A.values)
    st = cb.library_handle().cb_spmv(h, 1.0, 16, 0.0, 32, None)
    assert st == cb.CB_ERROR_NOT_SUPPORTED
    st = cb.library_handle().cb_spmm(h, 0, 1.0, 16, 1, 0.0, 32, 1, None)
    assert st in (cb.CB_ERROR_NOT_SUPPORTED, cb.CB_ERROR_INVALID_VALUE)
    cb.cb_destroy(h)
    assert cb.library_handle().cb_destroy(None) == cb.CB_SUCCESS
    assert cb.library_handle().cb_spmv(None, 1.0, 16, 0.0, 32, None) == cb.CB_ERROR_INVALID_VALUE


def test_copy_probe_validates_arguments():
    lib = cb.library_handle()
    assert lib.cb_copy_probe(16, 4096, 17, None) == cb.CB_ERROR_INVALID_VALUE
    assert lib.cb_copy_probe(16, 32, 64, None) == cb.CB_ERROR_INVALID_VALUE  # overlap
    assert lib.cb_copy_probe(None, 32, 64, None) == cb.CB_ERROR_INVALID_VALUE
    assert lib.cb_copy_probe(16, 32, 0, None) == cb.CB_SUCCESS


def test_read_probe_validates_arguments():
    lib = cb.library_handle()
    assert lib.cb_read_probe(16, 17, 4096, None) == cb.CB_ERROR_INVALID_VALUE
    assert lib.cb_read_probe(8, 64, 4096, None) == cb.CB_ERROR_INVALID_VALUE  # misaligned source
    assert lib.cb_read_probe(16, 64, None, None) == cb.CB_ERROR_INVALID_VALUE
    assert lib.cb_read_probe(16, -16, 4096, None) == cb.CB_ERROR_INVALID_VALUE
    assert lib.cb_read_probe(16, 0, 4096, None) == cb.CB_SUCCESS


@settings(max_examples=40, deadline=None)
@given(m=st.integers(0, 60), n=st.integers(0, 60), dens=st.floats(0, 1), seed=st.integers(0, 10 ** 6),
       vtype=st.sampled_from(["f64", "f32", "bf16"]), agg=st.sampled_from([-1, 0, 1]),
       th=st.sampled_from([(32, 128), (4, 40), (1, 1)]), lb=st.sampled_from(["contiguous", "paper", "none"]),
       tile_dim=st.sampled_from([16, 8]))
def test_random_round_trip(m, n, dens, seed, vtype, agg, th, lb, tile_dim):
    rng = np.random.default_rng(seed)
    D = np.where(rng.random((m, n)) < dens,
                 rng.choice([0.0, -0.0, np.nan, np.inf, 1.0, -2.5, 1e-40, 7e38], (m, n)) * 1.0, 0.0)
    keep = rng.random((m, n)) < dens
    A = matgen.from_dense(D, keep_zeros_mask=keep)
    roundtrip(A, vtype, col_agg=agg, th1=th[0], th2=th[1], lb_mode=lb, wave_nnz=int(rng.integers(0, 300)),
              tile_dim=tile_dim)
    if m * n <= 900 and vtype == "f64":
        check_against_model(A, col_agg=agg, th1=th[0], th2=th[1], lb=lb, tile_dim=tile_dim)


def test_automatic_range_size():
    """The automatic work per range: about 5120 ranges, none below 256 non-zero equivalents, and none
    above about 18 KB of codes and values (2048 FP64 entries, 3686 FP32, 4096 BF16); panels heavier
    than twice the target are the only ranges allowed past it."""
    small = matgen.laplacian_2d(64)  # 20,224 non-zeros: the floor (256 in non-zeros plus a cost per tile)
    M = cb.CbMatrix.from_csr(small, device=False)
    i = M.info
    assert 100 <= i["wave_nnz_mean"] <= 256 and i["nwaves"] <= small.nnz // 100, (i["wave_nnz_mean"], i["nwaves"])
    M.close()
    big = matgen.block_3d(60, seed=1)  # 13.4 M non-zeros: the FP64 byte cap binds, the others do not
    caps = {"f64": 2048, "f32": 3686, "bf16": 4096}
    means = {}
    for vt, cap in caps.items():
        M = cb.CbMatrix.from_csr(big, device=False, value_type=vt)
        i = M.info
        means[vt] = i["wave_nnz_mean"]
        assert i["wave_nnz_mean"] <= cap and i["wave_nnz_max"] <= 2 * cap, (vt, i["wave_nnz_mean"], i["wave_nnz_max"])
        M.close()
    # FP64 entries (9 bytes) reach the cap, and get more, shorter ranges than FP32 (5 bytes) and BF16 (3)
    assert means["f64"] < means["f32"] == means["bf16"]
    # where the cap binds, the ranges of the last stretch shrink to the remaining work / 2560, down to
    # a quarter of the cap; the other ranges keep the target; not when each XCD takes an eighth of the
    # ranges (equal counts: shorter ranges would leave the last XCD less work)
    for vt, tapered, kw in (("f64", True, {}), ("f32", False, {}), ("f64", False, {"xcd_chunk": 0})):
        M = cb.CbMatrix.from_csr(big, device=False, value_type=vt, **kw)
        st = cb.cb_export_structure(M.handle)
        w = np.add.reduceat(st["tile_nnz"].astype(np.int64) + 8, st["wave_ptr"][:-1])
        rem = np.cumsum(w[::-1])[::-1]  # work from each range to the end
        head = w[rem > 2560 * caps[vt]]
        if tapered:
            tail = w[rem < 2560 * caps[vt] // 8]
            assert len(tail) > 100 and tail.mean() < 0.5 * head.mean(), (tail.mean(), head.mean())
            # cut at panel boundaries (a panel here is about 400): about a quarter of the cap, not less
            assert 0.6 * caps[vt] / 4 <= np.median(tail) <= caps[vt] / 4, np.median(tail)
        else:
            last = w[-len(w) // 8:]
            assert abs(last.mean() - w.mean()) < 0.05 * w.mean(), (last.mean(), w.mean())
        M.close()
    # min_wave_nnz raises the automatic floor (small matrices: fewer, longer ranges), the cap too when
    # above it; an explicit wave_nnz ignores it; negative values are refused
    M = cb.CbMatrix.from_csr(small, device=False, min_wave_nnz=1024)
    # (non-zeros per range: the target counts 8 per tile on top)
    assert 600 <= M.info["wave_nnz_mean"] <= 1100 and M.info["nwaves"] <= small.nnz // 600, M.info["wave_nnz_mean"]
    M.close()
    M = cb.CbMatrix.from_csr(big, device=False, min_wave_nnz=1024)
    assert M.info["wave_nnz_mean"] <= caps["f64"], M.info["wave_nnz_mean"]  # the byte cap still binds above 1024
    M.close()
    M = cb.CbMatrix.from_csr(small, device=False, min_wave_nnz=4096, wave_nnz=300)
    assert M.info["wave_nnz_mean"] <= 400
    M.close()
    with pytest.raises(cb.CbError) as e:
        cb.CbMatrix.from_csr(small, device=False, min_wave_nnz=-1)
    assert e.value.status == cb.CB_ERROR_INVALID_VALUE
    # an explicit wave_nnz overrides the rule
    M = cb.CbMatrix.from_csr(big, device=False, wave_nnz=500)
    assert M.info["wave_nnz_mean"] <= 600
    M.close()


def test_automatic_kernel_choice():
    """spmv_kernel = -1: the quad kernel (2) where tiles hold >= 32 entries on average in row runs of
    two or more, else the streaming kernel (0); Algorithm 2 structures have no natural-order kernel."""
    n = 16
    cols = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
    cols.sort(axis=1)
    A = matgen.Csr(n, n, np.arange(0, 2 * n + 1, 2, dtype=np.int64), cols.ravel().astype(np.int32), np.ones(2 * n))
    # the same pattern without its last entry: 31 entries in the one tile
    B = matgen.Csr(n, n, np.minimum(np.arange(0, 2 * n + 1, 2, dtype=np.int64), 2 * n - 1),
                   cols.ravel()[:-1].astype(np.int32), np.ones(2 * n - 1))
    P = matgen.Csr(n, n, np.arange(n + 1, dtype=np.int64), ((np.arange(n) * 5) % n).astype(np.int32), np.ones(n))
    cases = [(A, {}, 2), (A, {"value_type": "bf16"}, 2), (A, {"spmv_kernel": 0}, 0), (A, {"lb_mode": "paper"}, 0),
             (A, {"lb_mode": "none"}, 2), (B, {}, 0), (P, {}, 0), (A, {"tile_dim": 8}, 0)]
    for M_, kw, want in cases:
        M = cb.CbMatrix.from_csr(M_, device=False, **kw)
        assert M.info["spmv_kernel"] == want, (kw, M.info["spmv_kernel"])
        if want == 2:
            assert M.info["row_reduce"] in (0, 2)  # one copy: the quad kernel sums its runs itself
        M.close()


def test_automatic_xcd_mapping():
    """xcd_chunk = -1: runs of 16 ranges per XCD unless 5 % or more of the entries lie farther than
    n / 8 from the diagonal (then each XCD takes a contiguous eighth); explicit values are kept."""
    lap = matgen.laplacian_2d(40)
    M = cb.CbMatrix.from_csr(lap, device=False)
    assert M.info["xcd_chunk"] == 16
    M.close()
    # a permutation matrix reversing the order: nearly every entry is far from the diagonal
    n = 400
    R = matgen.Csr(n, n, np.arange(n + 1, dtype=np.int64), (n - 1 - np.arange(n)).astype(np.int32), np.ones(n))
    M = cb.CbMatrix.from_csr(R, device=False)
    assert M.info["xcd_chunk"] == 0
    M.close()
    for c in (0, 1, 7, 1024):
        M = cb.CbMatrix.from_csr(R, device=False, xcd_chunk=c)
        assert M.info["xcd_chunk"] == c
        M.close()
    for bad in (-2, 1 << 21):
        with pytest.raises(cb.CbError) as e:
            cb.CbMatrix.from_csr(lap, device=False, xcd_chunk=bad)
        assert e.value.status == cb.CB_ERROR_INVALID_VALUE


def _poisson_box(nx, ny, nz):
    """7-point operator on an nx x ny x nz grid (x fastest): neighbours 1, nx and nx ny rows apart."""
    import scipy.sparse as sp

    def lap(k):
        return sp.diags([-np.ones(k - 1), 2 * np.ones(k), -np.ones(k - 1)], [-1, 0, 1])

    A = (sp.kron(sp.eye(nz), sp.kron(sp.eye(ny), lap(nx))) + sp.kron(sp.eye(nz), sp.kron(lap(ny), sp.eye(nx))) +
         sp.kron(lap(nz), sp.eye(nx * ny))).tocsr()
    A.sort_indices()
    return matgen.Csr(A.shape[0], A.shape[1], A.indptr.astype(np.int64), A.indices.astype(np.int32),
                      A.data.astype(np.float64))


def _tile_bases(st, info):
    """Each tile's column base: tile_cbase (cols16 1) or its quad batch header's fourth word (2)."""
    if info["cols16"] == 1:
        return st["tile_cbase"].astype(np.int64)
    bs = st["batch_stream"].reshape(-1, 4)
    base = np.empty(info["ntiles"], np.int64)
    for w in range(info["nwaves"]):
        t, o = st["wave_ptr"][w], st["batch_ptr"][w]
        while o < st["batch_ptr"][w + 1]:
            nt = bs[o, 1] & 0xFF
            base[t:t + nt] = bs[o, 3]
            t += nt
            o += 1 + nt
    return base


def test_compressed_tile_columns():
    """cols16: where every quad batch's original columns span less than 65,536, the quad kernel reads
    2-byte offsets from its batch's lowest column (kept in the batch header); otherwise, and for the
    streaming kernel, where every tile's columns span less than 65,536, 2-byte offsets from a 4-byte base
    per tile.  Decoded, they are the tile's columns (tile_cols), padding columns at offset 0; the
    structure counts 2 S (per batch) or 2 S + 4 (per tile) bytes per tile instead of 4 S.  Scattered
    far columns (power-law rows), no aggregation, Algorithm 2's tile-at-a-time order and cols16 = -1
    keep 4-byte columns."""
    box = _poisson_box(200, 200, 3)  # planes 40,000 rows apart: tiles span little, batches of 4 panels more
    for A, S, kern, want in ((matgen.block_3d(12, seed=3), 16, 2, 2), (matgen.poisson_3d(24), 16, 0, 1),
                             (matgen.poisson_3d(24), 8, 0, 1), (matgen.laplacian_2d(64), 16, 0, 1),
                             (matgen.poisson_3d(24), 16, 2, 2), (box, 16, 2, 1), (box, 16, 0, 1)):
        kw = {"col_agg": 1, "tile_dim": S, "cols16": 1, "spmv_kernel": kern}
        for lb in ("contiguous", "paper_stream") if S == 16 and kern == 2 else ("contiguous",):
            if lb == "paper_stream":
                kw = dict(kw, spmv_kernel=-1)
            M = cb.CbMatrix.from_csr(A, device=False, lb_mode=lb, **kw)
            i = M.info
            assert i["cols16"] == (want if lb == "contiguous" or A is not box else 1), (A.n, S, lb, i["cols16"])
            st = cb.cb_export_structure(M.handle)
            nt = i["ntiles"]
            cols = st["tile_cols"].reshape(nt, 4, S // 4).transpose(0, 2, 1).reshape(nt, S)  # natural order
            base = _tile_bases(st, i)
            dec = base[:, None] + st["tile_c16"].reshape(nt, S)
            p, c = st["tile_row"], st["tile_col"]
            first = st["cols_offset"][p] + S * c
            width = np.minimum(S, st["cols_offset"][p + 1] - first)
            real = np.arange(S)[None, :] < width[:, None]
            assert np.array_equal(dec[real], cols[real])
            assert np.all(st["tile_c16"].reshape(nt, S)[~real] == 0)
            if i["cols16"] == 1:
                assert np.array_equal(st["tile_cbase"], cols[:, 0])
            else:
                assert np.all(base <= cols[:, 0])
            M0 = cb.CbMatrix.from_csr(A, device=False, lb_mode=lb, **dict(kw, cols16=-1))
            assert M0.info["cols16"] == 0
            per_tile = 4 * S - 2 * S - (4 if i["cols16"] == 1 else 0)
            assert M0.info["spmv_bytes"] - i["spmv_bytes"] == per_tile * nt
            M0.close()
            M.close()
    for A, kw in ((matgen.power_law(100_000, seed=2), {}), (matgen.poisson_3d(24), {"col_agg": 0}),
                  (matgen.poisson_3d(24), {"col_agg": 1, "spmv_kernel": 1, "cols16": 1}),
                  (matgen.poisson_3d(24), {"col_agg": 1, "lb_mode": "paper"})):
        M = cb.CbMatrix.from_csr(A, device=False, **kw)
        assert M.info["cols16"] == 0, kw
        assert cb.cb_export_structure(M.handle)["tile_c16"].size == 0
        M.close()
    # automatic: a 2-byte form, except the per-tile one for the quad kernel with double vectors
    P = matgen.poisson_3d(24)
    for A, kw, want in ((P, {"spmv_kernel": 0}, 1), (P, {"spmv_kernel": 2}, 2), (box, {"spmv_kernel": 2}, 0),
                        (box, {"spmv_kernel": 2, "value_type": "f32"}, 1),
                        (box, {"spmv_kernel": 2, "value_type": "f32", "vector_f64": 1}, 0),
                        (box, {"lb_mode": "paper_stream"}, 0), (box, {"lb_mode": "paper_stream", "value_type": "bf16"}, 1),
                        (box, {"spmv_kernel": 2, "cols16": 1}, 1), (box, {"spmv_kernel": 0}, 1)):
        M = cb.CbMatrix.from_csr(A, device=False, col_agg=1, **kw)
        assert M.info["cols16"] == want, (A.n, kw, M.info["cols16"])
        M.close()
    # automatic kernel: with float vectors where the 2-byte form applies, the quad kernel (stencils
    # too); double vectors and scattered columns keep the streaming kernel on the stencil
    for A, kw, kern in ((P, {"value_type": "f32"}, 2), (P, {"value_type": "bf16"}, 2),
                        (P, {"value_type": "f32", "vector_f64": 1}, 0), (P, {}, 0),
                        (P, {"value_type": "f32", "cols16": -1}, 0),
                        (matgen.power_law(100_000, seed=2), {"value_type": "f32"}, 0)):
        M = cb.CbMatrix.from_csr(A, device=False, **kw)
        assert M.info["spmv_kernel"] == kern, kw
        M.close()
    for bad in (2, -2):
        with pytest.raises(cb.CbError) as e:
            cb.CbMatrix.from_csr(matgen.laplacian_2d(16), device=False, cols16=bad)
        assert e.value.status == cb.CB_ERROR_INVALID_VALUE


def test_quad_kernel_column_limit():
    # the quad kernel reads x at 32-bit byte offsets: 2^29 - 16 columns at most; beyond that the
    # explicit request and the streamed Algorithm 2 order (which runs it) are refused, and the
    # automatic choice takes the streaming kernel
    lim = (1 << 29) - 16
    for n, ok in ((lim, True), (lim + 1, False)):
        m = 64
        cols = np.stack([np.arange(m), n - 1 - np.arange(m)], 1).ravel().astype(np.int32)
        A = matgen.Csr(m, n, np.arange(0, 2 * m + 1, 2, dtype=np.int64), cols, np.ones(2 * m))
        for opts in ({"spmv_kernel": 2}, {"lb_mode": "paper_stream"}):
            if ok:
                M = host_matrix(A, **opts)
                assert M.info["spmv_kernel"] == 2
                M.close()
            else:
                with pytest.raises(cb.CbError, match="2\\^29"):
                    host_matrix(A, **opts)
        M = host_matrix(A)
        assert M.info["spmv_kernel"] == 0
        M.close()
