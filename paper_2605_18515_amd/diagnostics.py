"""Diagnostics and ablation settings on top of the C ABI (no arithmetic of the method here).

* ``ABLATION``: the option sets of the ablation in Section 4 (Fig. 12): CB-I keeps only the
  packing of each tile's data behind one virtual pointer (no column aggregation, one format,
  no load balance); CB-II adds column aggregation by the th0 rule and the per-tile format
  choice; the full method adds the inter-block load balance -- Algorithm 2 with the
  tile-at-a-time kernel of its scattered order, Algorithm 2's groups streamed (the packed tiles
  re-laid in group order, every tile's rows added with atomics), and the contiguous split this
  library defaults to.
* ``tile_nnz_histogram``: the non-zeros-per-tile histogram of Fig. 3 for a structure, from the
  tile counts the library exports.
* ``balance``: non-zeros per unit of work (Fig. 4's spread) as the library reports it.
"""
from __future__ import annotations

import numpy as np

from . import cbspmv as cb

ABLATION = {
    "CB-I": {"col_agg": 0, "th1": 257, "th2": 257, "lb_mode": "none"},
    "CB-II": {"col_agg": -1, "th1": 32, "th2": 128, "lb_mode": "none"},
    "CB (Alg. 2)": {"col_agg": -1, "th1": 32, "th2": 128, "lb_mode": "paper"},
    "CB (Alg. 2, streamed)": {"col_agg": -1, "th1": 32, "th2": 128, "lb_mode": "paper_stream"},
    "CB (contiguous)": {"col_agg": -1, "th1": 32, "th2": 128, "lb_mode": "contiguous"},
}

# Fig. 3's groups of tiles by non-zeros
HIST_EDGES = (1, 9, 17, 33, 65, 129, 257)
HIST_LABELS = ("1-8", "9-16", "17-32", "33-64", "65-128", "129-256")


def tile_nnz_histogram(M: "cb.CbMatrix") -> dict:
    """Tiles per non-zero group and their shares for the handle's structure (host or device)."""
    nnz = cb.cb_export_structure(M.handle)["tile_nnz"]
    counts, _ = np.histogram(nnz, bins=HIST_EDGES)
    total = int(nnz.size)
    return {"tiles": total, "counts": dict(zip(HIST_LABELS, map(int, counts))),
            "shares": dict(zip(HIST_LABELS, (float(c) / total if total else 0.0 for c in counts))),
            "share_1_32": float(counts[:3].sum()) / total if total else 0.0}


def balance(M: "cb.CbMatrix") -> dict:
    """Non-zeros per unit of work: Algorithm 2's groups and the kernel's wavefront ranges."""
    i = M.info
    return {k: i[k] for k in ("nquanta", "quantum_nnz_max", "quantum_nnz_mean", "quantum_nnz_std", "nwaves",
                              "wave_nnz_max", "wave_nnz_mean", "wave_nnz_std")}
