"""Diagnostics (tile histogram of Fig. 3, work balance of Fig. 4) and the ablation option sets,
host side: the library's tile counts against the oracle's plain partition, hand cases, and every
ablation setting converting to a valid structure."""
import numpy as np
import pytest

from oracle import cb_model
from paper_2605_18515_amd import cbspmv as cb
from paper_2605_18515_amd import diagnostics, matgen


def test_histogram_of_one_tile():
    M = cb.CbMatrix.from_csr(matgen.single_tile(5, seed=1), device=False)
    h = diagnostics.tile_nnz_histogram(M)
    M.close()
    assert h["tiles"] == 1 and h["counts"]["1-8"] == 1 and h["share_1_32"] == 1.0


@pytest.mark.parametrize("make", [lambda: matgen.block_3d(6, seed=1), lambda: matgen.poisson_3d(10),
                                  lambda: matgen.power_law(5000, seed=3, max_len=600, window=200)])
def test_histogram_matches_the_oracle_partition(make):
    A = make()
    M = cb.CbMatrix.from_csr(A, device=False, col_agg=0)
    h = diagnostics.tile_nnz_histogram(M)
    M.close()
    tiles = cb_model.plain_tiles(A.row_ptr, A.col_idx)
    nnz = np.array([len(v) for v in tiles.values()])
    want, _ = np.histogram(nnz, bins=diagnostics.HIST_EDGES)
    assert h["tiles"] == len(tiles) and list(h["counts"].values()) == list(map(int, want))
    assert abs(sum(h["shares"].values()) - 1.0) < 1e-12


def test_ablation_settings_convert_and_balance():
    A = matgen.power_law(20000, seed=2, max_len=3000, window=500)
    out = {}
    for name, opts in diagnostics.ABLATION.items():
        M = cb.CbMatrix.from_csr(A, device=False, **opts)
        out[name] = (M.info, diagnostics.balance(M))
        M.close()
    assert out["CB-I"][0]["col_agg"] == 0 and out["CB-I"][0]["tiles_csr"] == 0 and out["CB-I"][0]["tiles_dense"] == 0
    assert out["CB-II"][0]["col_agg"] == 1
    # Algorithm 2 balances its groups: no group heavier than the no-balance grouping's heaviest
    assert out["CB (Alg. 2)"][1]["quantum_nnz_std"] <= out["CB-II"][1]["quantum_nnz_std"]
    assert out["CB (Alg. 2)"][1]["quantum_nnz_max"] <= out["CB-II"][1]["quantum_nnz_max"]
