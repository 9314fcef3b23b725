"""Host-side checks of the quad kernel's batch records (spmv_kernel = 2; no GPU).

The converter cuts every work range into quad batches (format in
paper_2605_18515_amd/csrc/cb_stream.h).  These tests decode them independently
of the kernel and check (1) the limits the kernel relies on (16 tiles, 4
panels, 4 passes of 64 quads), (2) that the batches cover each work range's
tiles once and in order, and (3) that the kernel's own addressing -- the
tile of a lane found by a ballot over the tile-start marks, the code dword at
cb + 4 Q, the values at vb + 4 size(Val) Q, the entries present by lim or by
the Dense occupancy nibble, the payload read as zeros past its end -- applied
lane by lane on the CPU reproduces exactly the oracle's product on dyadic
inputs (every partial sum exact in FP64, whatever the order)."""
import numpy as np
import pytest

import oracle
from oracle import cb_model as cm
from paper_2605_18515_amd import matgen

cb = pytest.importorskip("paper_2605_18515_amd.cbspmv", reason="libcbspmv.so not built")

QT, QP, PANELS, PAD = 16, 3, 4, 2048
VSIZE = {"f64": 8, "f32": 4, "bf16": 2}


def aligned(b: int) -> int:
    """A tile region's bytes rounded to the 16-byte alignment of the next region."""
    return (b + cm.TILE_ALIGN - 1) // cm.TILE_ALIGN * cm.TILE_ALIGN


@np.errstate(invalid="ignore", over="ignore")
def values_of(raw: bytes, vtype):
    if vtype == "f64":
        return np.frombuffer(raw, np.float64).astype(np.float64)
    if vtype == "f32":
        return np.frombuffer(raw, np.float32).astype(np.float64)
    bits = np.frombuffer(raw, np.uint16).astype(np.uint32) << np.uint32(16)
    return bits.view(np.float32).astype(np.float64)


def emulate(A, X, vtype="f64", **opts):
    """y = A X computed from the exported quad batches exactly as the kernel addresses them.  With
    lb_mode paper_stream (Algorithm 2's groups streamed) the batches are in scatter form: any
    panels, the tile's position as its accumulator slot, its panel in the record."""
    M = cb.CbMatrix.from_csr(A, device=False, value_type=vtype, spmv_kernel=2, **opts)
    info, s = M.info, M.structure()
    M.close()
    assert info["spmv_kernel"] == 2
    scatter = info["lb_mode"] == cb.CB_LB_PAPER_STREAM
    vs = VSIZE[vtype]
    S = info["tile_dim"]  # tile size
    assert S == opts.get("tile_dim", 16)
    QPR = S // 4  # quads per Dense row
    agg = bool(info["col_agg"])
    pay = np.concatenate([s["payload"], np.zeros(PAD, np.uint8)])  # the readable padding reads zeros
    bs = s["batch_stream"].reshape(-1, 4)
    bp, wp = s["batch_ptr"], s["wave_ptr"]
    row, col, nnz, vp, ty = (s[k].astype(np.int64) for k in ("tile_row", "tile_col", "tile_nnz", "tile_vp",
                                                              "tile_type"))
    assert info["stream_bytes"] == 16 * (info["ntiles"] + info["nbatches"])
    y = np.zeros(A.m)
    seen = np.zeros(info["ntiles"], np.int64)  # entries multiplied per tile
    nb = 0
    for w in range(info["nwaves"]):
        o, oe = int(bp[w]), int(bp[w + 1])
        t0, t1 = int(wp[w]), int(wp[w + 1])
        if t0 == t1:
            assert o == oe
            continue
        B0 = int(vp[t0])

        def load(off, size):
            a = B0 + off
            out = np.zeros(size, np.uint8)
            for k in range(size):
                if 0 <= a + k < pay.size:
                    out[k] = pay[a + k]
            return out.tobytes()
        t = t0
        done_panels = []
        while o < oe:
            nb += 1
            h = bs[o]
            pb, hz, qtot = int(h[0]), int(h[1]), int(h[2])
            nt, npass, done = hz & 0xFF, (hz >> 8) & 0xFF, (hz >> 16) & 0xF
            recs = bs[o + 1:o + 1 + nt]
            tiles = list(range(t, t + nt))
            t += nt
            o += 1 + nt
            # limits
            assert 1 <= nt <= QT and 1 <= npass <= QP and npass == (qtot + 63) // 64 and qtot <= 64 * QP
            if scatter:
                assert pb == 0 and done == 0
                # the tiles of a range are packed back to back in kernel order
                for i in tiles[1:]:
                    assert vp[i] == vp[i - 1] + aligned(cm.tile_region_bytes(int(ty[i - 1]), int(nnz[i - 1]), vtype, S))
            else:
                assert row[tiles[0]] == pb and all(0 <= row[i] - pb < PANELS for i in tiles)
            quads = [S * S // 4 if ty[i] == cm.DENSE else (int(nnz[i]) + 3) // 4 for i in tiles]
            assert qtot == sum(quads)

            def fields(r):  # first quad, end of entries, slot
                meta = int(r[3])
                if scatter:
                    return (meta >> 5) & 0x3FF, (meta >> 16) & 0x1FFF, meta & 31
                return (meta >> 2) & 0x3FF, int(r[2]), meta & 3
            # marks and the ballot: the tile of every lane
            marks = np.zeros((QP, 64), bool)
            for r in recs:
                qs = fields(r)[0]
                marks[qs >> 6, qs & 63] = True
            jb = 0
            for p in range(npass):
                bal = marks[p]
                for lane in range(64):
                    below = int(bal[:lane].sum())
                    ti = jb + below + int(bal[lane]) - 1
                    r = recs[max(ti, 0)]
                    cbase, vbase, meta = int(r[0]), int(r[1]), int(r[3])
                    qs, lim, slot = fields(r)
                    q = 64 * p + lane
                    live = q < qtot
                    dense = live and ((meta >> 15) & 1)
                    i = tiles[max(ti, 0)]
                    if live and scatter:
                        assert slot == ti and int(r[2]) == row[i]
                    elif live:
                        assert slot == row[i] % PANELS
                    if dense:
                        dq = q - qs
                        assert 0 <= dq < S * S // 4
                        word = int.from_bytes(load(cbase + 4 * (dq >> 3), 4), "little")
                        vm = (word >> (4 * (dq & 7))) & 0xF
                        codes = [(((dq % QPR) << 6) | (dq // QPR)) + 16 * j for j in range(4)]
                    else:
                        nv = min(max(lim - 4 * q, 0), 4) if live else 0
                        vm = (1 << nv) - 1
                        codes = list(load(cbase + 4 * q, 4))
                    vals = values_of(load(vbase + 4 * vs * q, 4 * vs), vtype)
                    panel = int(r[2]) if scatter else pb + (slot - pb) % PANELS
                    for j in range(4):
                        if not (vm >> j) & 1:
                            continue
                        c = codes[j]
                        lc = c >> 4
                        assert lc < S and (c & 15) < S
                        if agg:
                            tc = s["tile_cols"][S * i:S * i + S].reshape(4, S // 4).T.ravel()
                            oc = int(tc[lc])
                        else:
                            oc = S * int(col[i]) + lc
                        y[S * panel + (c & 15)] += vals[j] * X[oc]
                        seen[i] += 1
                jb += int(bal.sum())
            for k in range(PANELS):
                if (done >> k) & 1:
                    done_panels.append(pb + k)
        assert t == t1
        if not scatter:
            assert sorted(done_panels) == sorted(set(row[t0:t1].tolist()))
    assert nb == info["nbatches"]
    assert np.array_equal(seen, nnz)
    return y


def dyadic_case(A, seed=7):
    rng = np.random.default_rng(seed)
    A = matgen.Csr(A.m, A.n, A.row_ptr, A.col_idx, rng.integers(-8, 9, A.nnz).astype(np.float64) / 8)
    return A, rng.integers(-8, 9, A.n).astype(np.float64) / 8


MATS = {
    "lap40": lambda: matgen.laplacian_2d(40),
    "block3": lambda: matgen.block_3d(3, seed=3),
    "poisson6": lambda: matgen.poisson_3d(6),
    "power": lambda: matgen.power_law(1500, seed=5, max_len=1000, window=150),
    "rect": lambda: matgen.random_csr(77, 203, 0.08, 4),
    "dense_mix": lambda: matgen.from_dense(
        np.where(np.random.default_rng(1).random((70, 90)) < np.repeat([0.95, 0.4, 0.05], [32, 20, 18])[:, None],
                 np.random.default_rng(2).uniform(-1, 1, (70, 90)), 0.0)),
}


@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("col_agg", [0, 1])
@pytest.mark.parametrize("name", sorted(MATS))
def test_quad_batches_decode_to_the_product(name, col_agg, vtype):
    A, X = dyadic_case(MATS[name]())
    assert np.array_equal(emulate(A, X, vtype, col_agg=col_agg), oracle.spmv(A, X))


@pytest.mark.parametrize("vtype", ["f64", "bf16"])
@pytest.mark.parametrize("col_agg", [0, 1])
@pytest.mark.parametrize("name", sorted(MATS))
def test_quad_batches_decode_to_the_product_8x8(name, col_agg, vtype):
    A, X = dyadic_case(MATS[name]())
    assert np.array_equal(emulate(A, X, vtype, col_agg=col_agg, tile_dim=8, th1=8, th2=40), oracle.spmv(A, X))


@pytest.mark.parametrize("th", [(32, 128), (1, 1), (300, 300), (4, 40)])
def test_quad_batches_every_format(th):
    A, X = dyadic_case(MATS["dense_mix"]())
    assert np.array_equal(emulate(A, X, "f64", th1=th[0], th2=th[1], col_agg=0), oracle.spmv(A, X))


@pytest.mark.parametrize("wave_nnz", [40, 300, 5000])
@pytest.mark.parametrize("lb", ["contiguous", "none"])
def test_quad_batches_follow_the_work_ranges(wave_nnz, lb):
    A, X = dyadic_case(matgen.power_law(2000, seed=8, max_len=1500, window=300))
    assert np.array_equal(emulate(A, X, "f64", lb_mode=lb, wave_nnz=wave_nnz, quantum_tiles=3),
                          oracle.spmv(A, X))


def test_quad_limits_cut_batches():
    # one panel of dense tiles: a Dense tile is 64 quads, so at most four per batch
    A, X = dyadic_case(matgen.from_dense(np.random.default_rng(3).uniform(-1, 1, (16, 640))))
    M = cb.CbMatrix.from_csr(A, device=False, col_agg=0, spmv_kernel=2)
    info = M.info
    M.close()
    assert info["tiles_dense"] == 40 and info["nbatches"] >= 10
    assert np.array_equal(emulate(A, X, "bf16", col_agg=0), oracle.spmv(A, X))
    # one tile per panel over many panels: the 4-panel limit cuts
    A2, X2 = dyadic_case(matgen.identity(16 * 40))
    assert np.array_equal(emulate(A2, X2, "f64"), oracle.spmv(A2, X2))


@pytest.mark.parametrize("vtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("col_agg", [0, 1])
@pytest.mark.parametrize("name", sorted(MATS))
def test_streamed_algorithm2_batches_decode_to_the_product(name, col_agg, vtype):
    """lb_mode paper_stream: Algorithm 2's groups, the packed tiles re-laid in group order, quad
    batches in scatter form; the kernel's addressing reproduces the product, every panel is
    pre-scaled (all shared), and the grouping is the paper mode's."""
    A, X = dyadic_case(MATS[name]())
    for wave_nnz in (0, 50):
        assert np.array_equal(emulate(A, X, vtype, col_agg=col_agg, lb_mode="paper_stream", wave_nnz=wave_nnz),
                              oracle.spmv(A, X))
    Ms = cb.CbMatrix.from_csr(A, device=False, value_type=vtype, col_agg=col_agg, lb_mode="paper_stream")
    Mp = cb.CbMatrix.from_csr(A, device=False, value_type=vtype, col_agg=col_agg, lb_mode="paper")
    ss, sp = Ms.structure(), Mp.structure()
    i_s, i_p = Ms.info, Mp.info
    Ms.close()
    Mp.close()
    for k in ("tile_ori", "quantum_ptr", "tile_row", "tile_col", "tile_nnz", "tile_type"):
        assert np.array_equal(ss[k], sp[k]), k
    assert i_s["payload_bytes"] == i_p["payload_bytes"] and i_s["prepass_panels"] == i_s["npanels"]
    assert i_s["quantum_nnz_std"] == i_p["quantum_nnz_std"]
    # the same packed tile regions, moved
    vs = VSIZE[vtype]
    for t in range(i_s["ntiles"]):
        rb = aligned(cm.tile_region_bytes(int(ss["tile_type"][t]), int(ss["tile_nnz"][t]), vtype, 16))
        a, b = int(ss["tile_vp"][t]), int(sp["tile_vp"][t])
        assert np.array_equal(ss["payload"][a:a + rb], sp["payload"][b:b + rb])


def test_streamed_algorithm2_options():
    A = matgen.laplacian_2d(20)
    for kw in ({"tile_dim": 8}, {"spmv_kernel": 0}, {"spmv_kernel": 1}):
        with pytest.raises(cb.CbError) as e:
            cb.CbMatrix.from_csr(A, device=False, lb_mode="paper_stream", **kw)
        assert e.value.status == cb.CB_ERROR_NOT_SUPPORTED
    M = cb.CbMatrix.from_csr(A, device=False, lb_mode="paper_stream", spmv_kernel=2)
    assert M.info["spmv_kernel"] == 2 and M.info["lb_mode"] == cb.CB_LB_PAPER_STREAM
    rp, ci, va = M.export_csr()
    M.close()
    assert np.array_equal(rp, A.row_ptr) and np.array_equal(ci, A.col_idx)
    assert np.array_equal(va.view(np.uint64), A.values.view(np.uint64))
