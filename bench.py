#!/usr/bin/env python3
"""Benchmark of the CB-SpMV hot path on one MI355X.

Workload: FP64 y = A*x on the 3D block matrix -- 7-point adjacency on a
100^3 grid, 3 unknowns per node as dense 3x3 blocks of U[-1,1] values with 10
added on the scalar diagonal (n = 3,000,000, nnz = 62,460,000), x ~ U[-1,1],
alpha = 1, beta = 0.  The matrix is converted once (timed separately, host
converter + one upload); a step is one cb_spmv over the resident structure.

Prints ONE JSON line with the throughput (GFLOP/s = 2*nnz/t), the HBM roofline
of the SpMV kernel (algorithmic bytes of the built structure + x + y per launch,
over the kernel time from HIP events on the launch stream), the CPU oracle's
rate on the same matrix, and the mixed-precision / k-right-hand-side legs.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SpMV GFLOP/s & % HBM roofline (FP64 vs mixed); batched solves/s, p50/p99"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_spmv_f64_block3d.json")


WORKLOADS = {
    "block3d": "FP64 y=A*x, 3D block matrix {side}^3 grid x 3 dof (7-point, dense 3x3 blocks, diag +10)",
    "powerlaw": "FP64 y=A*x, power-law rows: n=4,000,000, Zipf(2.1) lengths in [1,1e5] scaled to mean 16, "
                "70% of columns within +-2048 of the diagonal",
    "powerlaw_literal": "FP64 y=A*x, power-law rows: n=4,000,000, Zipf(2.1) lengths in [1,1e5] unscaled (mean 4.8), "
                        "70% of columns within +-2048 of the diagonal",
    "poisson": "FP64 y=A*x, 3D 7-point Poisson operator on a 192^3 grid",
    "laplacian": "FP64 y=A*x, 2D 5-point Laplacian on a 64x64 grid",
}


def make_matrix(name: str, side: int):
    from paper_2605_18515_amd import matgen

    if name == "block3d":
        return matgen.block_3d(side, 3, 10.0, seed=1)
    if name == "powerlaw":
        return matgen.power_law(4_000_000, seed=2)
    if name == "powerlaw_literal":
        return matgen.power_law(4_000_000, seed=2, mean_len=None)
    if name == "poisson":
        return matgen.poisson_3d(192)
    return matgen.laplacian_2d(64)


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """sha256[:16] of the kernel source with comments and blank lines removed, so the committed
    counters stay valid across comment edits and go stale on any code change."""
    code = []
    with open(os.path.join(ROOT, "paper_2605_18515_amd", "csrc", "kernels.hip")) as f:
        for line in f:
            line = line.split("//", 1)[0].rstrip()
            if line:
                code.append(line)
    return hashlib.sha256("\n".join(code).encode()).hexdigest()[:16]


def measured_traffic(nnz: int, spmv_bytes: int):
    """HBM bytes per launch from the committed rocprofv3 counter runs, when they were taken on the
    current kernel source and on this structure (the same non-zeros and algorithmic bytes)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if t.get("nnz") != nnz or t.get("spmv_bytes") != spmv_bytes:
        return None
    return t.get("bytes_per_launch")


def time_graph(fn, steps: int, warmup: int, replays: int = 5):
    """Capture `steps` calls in one HIP graph (torch's capture stream) and time
    its replays: per-launch time without host launch overhead."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(steps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(replays):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall / (steps * replays), e0.elapsed_time(e1) / 1e3 / (steps * replays)


def kernel_name(info: dict, lb: str) -> str:
    """The product kernel a handle launches (value type FP64), as the trace names it with its template
    arguments spelled out."""
    if lb == "paper":
        return "spmv_kernel<FP64> (Algorithm 2 order)"
    if lb == "paper_stream":
        agg = "aggregated" if info["col_agg"] else "plain columns"
        return f"spmv_quad_kernel<FP64, {agg}, row sums {info['row_reduce']}, scatter> (Algorithm 2 order, streamed)"
    agg = "aggregated" if info["col_agg"] else "plain columns"
    if info["col_agg"] and info.get("cols16"):
        agg += ", 2-byte column offsets per " + ("batch" if info["cols16"] == 2 else "tile")
    if info["spmv_kernel"] == 1:
        return f"spmv_rows_kernel<FP64, {agg}>"
    if info["spmv_kernel"] == 2:
        return f"spmv_quad_kernel<FP64, {agg}, row sums {info['row_reduce']}>"
    return f"spmv_stream_kernel<FP64, {agg}, row sums {info['row_reduce']}>"


def time_calls(fn, steps: int, warmup: int):
    import torch

    for _ in range(warmup):
        fn()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall / steps, e0.elapsed_time(e1) / 1e3 / steps


STORAGE_TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2}


def settle(fn, seconds: float):
    """Untimed launches of fn for at least `seconds` of wall time, synchronising every 16 launches:
    the GPU leaves its idle clocks within milliseconds to tens of milliseconds of sustained work, so
    a short timed window right after host-side work would otherwise measure part of that ramp.
    Returns (launches, seconds)."""
    import torch

    n, t0 = 0, time.perf_counter()
    while True:
        for _ in range(16):
            fn()
        n += 16
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if el >= seconds:
            return n, el


def gpu_sclk():
    """The shader clock level the driver reports as current (sysfs pp_dpm_sclk, the line marked
    '*'), or None where it is not readable."""
    import glob

    for f in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
        try:
            with open(f) as fh:
                for line in fh:
                    if line.rstrip().endswith("*"):
                        return line.split(":", 1)[-1].replace("*", "").strip()
        except OSError:
            continue
    return None


def rows_of(A, rows):
    """The sub-matrix of the given rows (same columns): its oracle product is exactly those rows."""
    import numpy as np

    from paper_2605_18515_amd import matgen

    rows = np.asarray(rows)
    starts, ends = A.row_ptr[rows], A.row_ptr[rows + 1]
    idx = np.concatenate([np.arange(s, e) for s, e in zip(starts, ends)]) if rows.size else np.zeros(0, np.int64)
    rp = np.concatenate([[0], np.cumsum(ends - starts)]).astype(np.int64)
    return matgen.Csr(rows.size, A.n, rp, A.col_idx[idx], A.values[idx])


def sample_rows(A, count: int, seed: int):
    """A seeded sample of rows, plus the first, the last and the longest ones."""
    import numpy as np

    lens = np.diff(A.row_ptr)
    pick = np.random.default_rng(seed).choice(A.m, min(count, A.m), replace=False)
    return np.unique(np.concatenate([pick, np.argsort(lens)[-16:], [0, A.m - 1]]))


def spmv_leg(cb, A, dev, steps: int, settle_s: float, check: bool, workload: str, **opts) -> dict:
    """FP64 SpMV of A (default options: the paper's rules, contiguous ranges), x from seed 1: kernel
    time from HIP events over `steps` launches after an untimed settle, algorithmic bytes and their
    fraction of the HBM peak, and the max scaled error of every row against the oracle."""
    import numpy as np
    import torch

    from paper_2605_18515_amd import matgen

    x = matgen.vector(A.n, 1)
    M = cb.CbMatrix.from_csr(A, **opts)
    info = M.info
    xd = torch.from_numpy(x).to(dev)
    yd = torch.empty(A.m, dtype=torch.float64, device=dev)
    step = lambda: M.spmv(xd, yd)  # noqa: E731
    settle(step, settle_s)
    wall, kern = time_calls(step, steps, 0)
    leg = {"workload": workload, "n": A.n, "nnz": A.nnz, "kernel_us": kern * 1e6, "gflops": 2.0 * A.nnz / wall / 1e9,
           "spmv_bytes": info["spmv_bytes"], "GBs": info["spmv_bytes"] / kern / 1e9,
           "frac": info["spmv_bytes"] / kern / 1e9 / HBM_PEAK_GBS, "col_agg": info["col_agg"],
           "row_reduce": info["row_reduce"], "nwaves": info["nwaves"], "shared_panels": info["shared_panels"],
           "kernel": kernel_name(info, "contiguous")}
    if check:
        import oracle

        y = yd.cpu().numpy()
        e, viol, _ = oracle.scaled_error(y, oracle.spmv(A, x, comp=True), oracle.scale(A, x), 1e-12)
        leg["max_scaled_error"] = e
        leg["violations"] = viol
        if viol:
            raise RuntimeError(f"{workload}: {viol} rows outside the 1e-12 tolerance (max {e})")
    M.close()
    del xd, yd
    return leg


def laplacian_leg(cb, dev, check: bool) -> dict:
    """The 64 x 64 five-point Laplacian (20,224 non-zeros, cache-resident): latency of one SpMV
    launched on its own, and per launch when 1000 launches replay as one captured HIP graph."""
    import torch

    from paper_2605_18515_amd import matgen

    A = matgen.laplacian_2d(64)
    x = matgen.vector(A.n, 1)
    M = cb.CbMatrix.from_csr(A)
    xd = torch.from_numpy(x).to(dev)
    yd = torch.empty(A.m, dtype=torch.float64, device=dev)
    step = lambda: M.spmv(xd, yd)  # noqa: E731
    settle(step, 0.2)
    w1, k1 = time_calls(step, 1000, 0)
    wg, kg = time_graph(step, 1000, 10)
    leg = {"workload": WORKLOADS["laplacian"], "nnz": A.nnz, "stream_launch_us": w1 * 1e6,
           "stream_kernel_us": k1 * 1e6, "graph_replay_us_per_launch": kg * 1e6,
           "graph_gflops": 2.0 * A.nnz / kg / 1e9, "spmv_bytes": M.info["spmv_bytes"],
           "note": "working set in cache: launch-bound, not an HBM roofline figure"}
    if check:
        import oracle

        e, viol, _ = oracle.scaled_error(yd.cpu().numpy(), oracle.spmv(A, x, comp=True), oracle.scale(A, x), 1e-12)
        leg["max_scaled_error"] = e
        if viol:
            raise RuntimeError(f"laplacian: {viol} rows outside the 1e-12 tolerance (max {e})")
    M.close()
    return leg


CG_LEGS = ("fp64_cg", "replace_f32", "replace_bf16", "replace_f32w", "replace_bf16w", "restart_f32", "restart_bf16",
           "restart_f32w")


def cg_legs(args, cb, matgen, names=CG_LEGS):
    """Solves of A x = b from x = 0 on the 192^3 Poisson operator (b ~ U[-1, 1]) until the FP64
    residual |b - A x| / |b| is at most 1e-10: FP64 CG, and the two mixed-precision solvers
    (residual replacement and restarted refinement) with the products on the FP32 and on the BF16
    copy of A.  Each solve is timed whole (host polling included).  Returns (legs, A, ok)."""
    import numpy as np
    import torch

    rtol = 1e-10
    A = matgen.poisson_3d(192)
    b = matgen.vector(A.n, 5)
    bd = torch.from_numpy(b).to("cuda")
    M = cb.CbMatrix.from_csr(A, value_type="f64")
    legs = {}
    xs = {}
    # <method>_<storage>[w]: w = double vectors on the low-precision copy
    for name in names:
        vt = name.split("_")[-1]
        L = None if name == "fp64_cg" else cb.CbMatrix.from_csr(A, value_type=vt.rstrip("w"),
                                                                 vector_f64=int(vt.endswith("w")))
        meth = cb.CB_REFINE_RESTART if name.startswith("restart") else cb.CB_REFINE_REPLACE
        xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        work = torch.empty(cb.cb_cg_workspace_bytes(M.handle, L.handle if L else None), dtype=torch.uint8,
                           device="cuda")
        solve = (lambda: M.cg(bd, xd, work, rtol=rtol)) if L is None else \
            (lambda: M.cg_refine(L, bd, xd, work, rtol=rtol, refine_method=meth))
        times = []
        for rep in range(1 + max(1, min(args.steps, 5))):
            xd.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = solve()
            torch.cuda.synchronize()
            if rep:  # the first solve is warm-up
                times.append(time.perf_counter() - t0)
        sec = float(np.median(times))
        legs[name] = {"solves_per_s": 1.0 / sec, "seconds": sec, "iterations": res["iterations"],
                      "refinements": res["refinements"], "restarts": res["restarts"],
                      "rel_residual_device": res["rel_residual"],
                      "converged": res["converged"]}
        xs[name] = xd.cpu().numpy()
        log(f"{name}: {json.dumps(legs[name])}")
        if L is not None:
            L.close()
        del work, xd
        torch.cuda.empty_cache()
    M.close()
    ok = True
    if not args.no_check:
        from oracle import solvers

        for name, x in xs.items():
            legs[name]["rel_residual_oracle"] = r = solvers.residual(A, b, x)
            ok = ok and r <= rtol and legs[name]["converged"]
        log("oracle residuals: " + ", ".join(f"{k} {v['rel_residual_oracle']:.3e}" for k, v in legs.items()))
    return legs, A, ok


def run_cg(args, cb, matgen) -> int:
    legs, A, ok = cg_legs(args, cb, matgen)
    best = max(legs, key=lambda k: legs[k]["solves_per_s"])
    out = {
        "metric": "CG solves/s to |b - Ax| / |b| <= 1e-10 (FP64 vs mixed-precision refinement)",
        "value": round(legs[best]["solves_per_s"], 4), "unit": "solves/s", "n_gpus": 1,
        "steps": max(1, min(args.steps, 5)), "warmup": 1, "ms_per_step": legs[best]["seconds"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "CG on the 3D 7-point Poisson operator, 192^3 grid, b ~ U[-1,1], x0 = 0",
                   "n": A.n, "nnz": A.nnz, "method": best},
        "roofline": None, "cpu_baseline": None,
        "extra": {"legs": legs, "speedup_vs_fp64_cg": {k: legs[k]["solves_per_s"] / legs["fp64_cg"]["solves_per_s"]
                                                       for k in legs}},
    }
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


def _serve_matrix(spec):
    """One resident matrix of the serving workload: (family, n, seed) -> Csr."""
    from paper_2605_18515_amd import matgen

    fam, n, seed = spec
    if fam == "block3d":
        return matgen.block_3d(max(2, round((n / 3) ** (1 / 3))), 3, 10.0, seed=seed)
    if fam == "powerlaw":
        return matgen.power_law(n, seed=seed, max_len=min(100_000, max(16, n // 4)))
    return matgen.poisson_3d(max(2, round(n ** (1 / 3))))


def serve_legs(args, cb, matgen, nreq: int) -> dict:
    """Serving workload: 256 resident matrices from the three families (3D block, power-law, 3D
    Poisson) with n log-uniform in [1e3, 1e6], every other one stored in FP32; requests are SpMM
    with k uniform in 1..16 on any matrix, or a CG solve (cap 500 iterations) on a Poisson matrix to
    a relative residual of 1e-10, half each: on a FP64 matrix plain CG, on a FP32 one the refined
    kind (the FP32 copy's products, FP64 residual replacement with a FP64 twin of the matrix; only
    a true residual ends it).  Three runs of the same request list: the server with every request
    submitted at once (throughput), the server under Poisson arrivals at a quarter, half and all of
    that rate (p50/p99 latency against load), and the plain path, one request at a time through cb_spmm, cb_cg and cb_cg_refine.
    Then the precision comparison on the Poisson matrices alone (serve_precision).  Returns the
    measurements."""
    import multiprocessing as mp

    import numpy as np
    import torch

    rng = np.random.default_rng(2026)
    fams = ("block3d", "powerlaw", "poisson")
    specs = [(fams[i % 3], int(round(10 ** rng.uniform(3, 6))), 100 + i) for i in range(256)]
    t = time.perf_counter()
    with mp.get_context("fork").Pool(8) as pool:
        csrs = pool.map(_serve_matrix, specs)
    log(f"generated 256 matrices ({sum(A.nnz for A in csrs) / 1e6:.0f} M non-zeros) in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    sw = {"min_wave_nnz": args.serve_min_wave_nnz}
    # --serve-tune: one cb_tune per (family, value type) on the family's largest matrix; its structural choices
    # (aggregation, sub-block size, kernel, column form, thresholds, row sums, split, XCD mapping) go to every
    # handle of that family and type, the range size stays automatic (it depends on the matrix's size)
    tuned = {}
    if args.serve_tune:
        t = time.perf_counter()
        for fam in fams:
            idx = [i for i, sp in enumerate(specs) if sp[0] == fam]
            for vt in ("f64", "f32"):
                big = max((i for i in idx if (i % 2 == 0) == (vt == "f64")), key=lambda i: csrs[i].nnz)
                _, best, _ = cb.cb_tune(csrs[big], keep=False, value_type=vt, **sw)
                best = {k: v for k, v in best.items() if k not in ("wave_nnz", "value_type", "host_threads")}
                tuned[(fam, vt)] = best
        log(f"tuned the serving handles' options in {time.perf_counter() - t:.1f}s: " +
            "; ".join(f"{f} {v}: S={o['tile_dim']} k{o['spmv_kernel']} agg={o['col_agg']} th=({o['th1']},{o['th2']}) "
                      f"rr={o['row_reduce']} lb={o['lb_mode']} xcd={o['xcd_chunk']} c16={o['cols16']}"
                      for (f, v), o in tuned.items()))

    def hopts(i, vt):
        return dict(sw, **tuned.get((specs[i][0], vt), {}))

    mats = [cb.CbMatrix.from_csr(A, value_type="f64" if i % 2 == 0 else "f32", **hopts(i, "f64" if i % 2 == 0 else "f32"))
            for i, A in enumerate(csrs)]
    dts = [np.float64 if i % 2 == 0 else np.float32 for i in range(256)]
    spd = [i for i, s in enumerate(specs) if s[0] == "poisson"]
    # FP64 twins of the FP32 Poisson matrices: the refined solves' residual replacement
    twin = {i: cb.CbMatrix.from_csr(csrs[i], **hopts(i, "f64")) for i in spd if dts[i] == np.float32}
    log(f"converted and uploaded in {time.perf_counter() - t:.1f}s, "
        f"{sum(M.info['device_bytes'] for M in list(mats) + list(twin.values())) / 2 ** 30:.2f} GiB on the device")
    # inputs: one random block per matrix (X = its first n * k values), b per Poisson matrix (double
    # for the refined solves)
    xin = [np.random.default_rng(i).uniform(-1, 1, A.n * 16).astype(dts[i]) for i, A in enumerate(csrs)]
    b64 = {i: xin[i][:csrs[i].n].astype(np.float64) for i in twin}
    reqs = []
    for r in range(nreq):
        if rng.random() < 0.5:
            i = int(rng.choice(spd))
            reqs.append(("cg", i, 1))
        else:
            reqs.append(("spmm", int(rng.integers(0, 256)), int(rng.integers(1, 17))))
    rtol, cap = 1e-10, 500

    def outputs():
        return [np.zeros(csrs[i].n * k, dts[i]) if kind == "spmm" else
                np.zeros(csrs[i].n, np.float64 if i in twin else dts[i]) for kind, i, k in reqs]

    def submit_all(S, ids, outs, gaps=None, count=None):
        tickets = []
        for j, (kind, i, k) in enumerate(reqs[:count]):
            if gaps is not None:
                time.sleep(gaps[j])
            if kind == "cg" and i in twin:
                tickets.append(S.submit_cg_refine(ids[("hi", i)], i, b64[i], outs[j], rtol=rtol, max_iter=cap))
            elif kind == "cg":
                tickets.append(S.submit_cg(i, xin[i][:csrs[i].n], outs[j], rtol=rtol, max_iter=cap))
            else:
                tickets.append(S.submit_spmm(i, xin[i][:csrs[i].n * k].reshape(csrs[i].n, k),
                                             outs[j].reshape(csrs[i].m, k)))
        return tickets

    max_active, arena = args.serve_active, args.serve_arena_gib

    def serve(gaps=None, count=None):
        outs = outputs()
        S = cb.CbServer(max_active=max_active, arena_bytes=arena << 30)
        ids = {i: S.add_matrix(M) for i, M in enumerate(mats)}
        ids.update({("hi", i): S.add_matrix(M) for i, M in twin.items()})
        tickets = submit_all(S, ids, outs, gaps, count)
        resp = [S.wait(t) for t in tickets]
        st = S.stats()
        S.close()
        return outs, resp, st

    serve(count=64)  # warm-up: code objects, arena, graphs
    outs_b, resp_b, st_b = serve()
    log(f"server, all at once: {st_b['requests_per_s']:.0f} requests/s, {st_b['solves_per_s']:.1f} solves/s, "
        f"p50 {st_b['p50_us'] / 1e3:.2f} ms, p99 {st_b['p99_us'] / 1e3:.2f} ms, active peak {st_b['active_peak']}")
    # Poisson arrivals at fractions of the saturated request rate: latency against load
    sweep = []
    for frac in (0.25, 0.5, 1.0):
        lam_f = frac * st_b["requests_per_s"]
        gaps = np.random.default_rng(7).exponential(1.0 / lam_f, len(reqs))
        _, _, st_f = serve(gaps)
        sweep.append({"load": frac, "rate_per_s": lam_f, "requests_per_s": st_f["requests_per_s"],
                      "solves_per_s": st_f["solves_per_s"], "p50_ms": st_f["p50_us"] / 1e3,
                      "p99_ms": st_f["p99_us"] / 1e3})
        log(f"server, Poisson arrivals at {lam_f:.0f}/s ({frac:.2f} of saturation): {st_f['requests_per_s']:.0f} "
            f"requests/s, p50 {st_f['p50_us'] / 1e3:.2f} ms, p99 {st_f['p99_us'] / 1e3:.2f} ms")
        if frac == 0.5:
            lam, st_p = lam_f, st_f

    # the plain path: one request at a time
    dev = torch.device("cuda:0")
    lat = []
    t0 = time.perf_counter()
    outs_s = outputs()
    for j, (kind, i, k) in enumerate(reqs):
        ts = time.perf_counter()
        M, A, tdt = mats[i], csrs[i], torch.float64 if dts[i] == np.float64 else torch.float32
        if kind == "cg" and i in twin:
            x = torch.zeros(A.n, dtype=torch.float64, device=dev)
            twin[i].cg_refine(M, torch.from_numpy(b64[i]).to(dev), x, rtol=rtol, max_iter=cap, check_every=8)
            outs_s[j][:] = x.cpu().numpy()
        elif kind == "cg":
            b = torch.from_numpy(xin[i][:A.n]).to(dev)
            x = torch.zeros(A.n, dtype=tdt, device=dev)
            M.cg(b, x, rtol=rtol, max_iter=cap, check_every=8)
            outs_s[j][:] = x.cpu().numpy()
        else:
            X = torch.from_numpy(xin[i][:A.n * k]).to(dev).reshape(A.n, k)
            Y = torch.zeros((A.m, k), dtype=tdt, device=dev)
            M.spmm(X, Y)
            outs_s[j][:] = Y.cpu().numpy().ravel()
        lat.append(time.perf_counter() - ts)
    el = time.perf_counter() - t0
    ncg = sum(1 for r in reqs if r[0] == "cg")
    seq = {"requests_per_s": len(reqs) / el, "solves_per_s": ncg / el, "p50_ms": float(np.percentile(lat, 50)) * 1e3,
           "p99_ms": float(np.percentile(lat, 99)) * 1e3}
    log(f"one at a time: {seq['requests_per_s']:.0f} requests/s, {seq['solves_per_s']:.1f} solves/s")
    # the served results against the plain path's
    worst = 0.0
    for j, (kind, i, k) in enumerate(reqs):
        a, b_ = outs_b[j].astype(np.float64), outs_s[j].astype(np.float64)
        worst = max(worst, float(np.abs(a - b_).max() / max(1e-300, np.abs(b_).max())))
    conv = sum(1 for (kind, _, _), r in zip(reqs, resp_b) if kind == "cg" and r["converged"])
    nref = sum(1 for kind, i, _ in reqs if kind == "cg" and i in twin)
    for M in mats + list(twin.values()):
        M.close()
    del mats, twin
    torch.cuda.empty_cache()
    prec = serve_precision(args, cb, [csrs[i] for i in spd], [xin[i] for i in spd],
                           {vt: tuned.get(("poisson", "f64" if vt == "f64" else "f32"), {}) for vt in ("f64", "f32", "bf16")})
    return {"requests": len(reqs), "cg_requests": ncg, "refined_requests": nref, "rtol": rtol, "all_at_once": st_b,
            "poisson_arrivals": dict(st_p, rate_per_s=lam), "arrival_sweep": sweep, "one_at_a_time": seq,
            "speedup_solves_vs_one_at_a_time": st_b["solves_per_s"] / seq["solves_per_s"],
            "cg_converged": conv, "max_rel_diff_vs_one_at_a_time": worst, "precision": prec,
            "tuned_options": {f"{f}_{v}": o for (f, v), o in tuned.items()} or None}


def serve_precision(args, cb, csrs, xin, tuned=None, nsolves: int = 256) -> dict:
    """FP64 serving against mixed-precision serving at the same accuracy: the serving workload's
    Poisson matrices, each resident as FP64, FP32 and BF16 handles; the same nsolves CG requests
    (random matrix, b from the matrix's input block, x0 = 0, cap 500 iterations) served all at once
    three ways -- plain FP64 CG (recurrence residual <= 1e-10), and the refined kind on the BF16 and
    on the FP32 copy (FP64 residual replacement, true residual <= 1e-10).  Every solve's true
    residual is then measured with the CPU oracle on a sample."""
    import numpy as np

    import oracle  # noqa: F401  (the oracle's true residual)
    from oracle import solvers

    rng = np.random.default_rng(77)
    pick = [int(rng.integers(0, len(csrs))) for _ in range(nsolves)]
    H = {}
    for vt in ("f64", "f32", "bf16"):
        H[vt] = [cb.CbMatrix.from_csr(A, value_type=vt, **dict((tuned or {}).get(vt, {}),
                                                                min_wave_nnz=args.serve_min_wave_nnz)) for A in csrs]
    bs = [xin[i][:csrs[i].n].astype(np.float64) for i in range(len(csrs))]
    out = {"workload": f"{len(csrs)} resident 3D Poisson matrices (n log-uniform in [1e3, 1e6]), {nsolves} CG "
                       "solves to 1e-10, x0 = 0, cap 500 iterations, all submitted at once", "solves": nsolves}
    check = sorted(set(int(j) for j in rng.choice(nsolves, min(24, nsolves), replace=False)))
    for mode in ("fp64_cg", "refine_bf16", "refine_f32"):
        S = cb.CbServer(max_active=args.serve_active, arena_bytes=args.serve_arena_gib << 30)
        ids = {vt: [S.add_matrix(M) for M in H[vt]] for vt in H}
        xs = [np.zeros(csrs[i].n) for i in pick]
        tickets = []
        for j, i in enumerate(pick):
            if mode == "fp64_cg":
                tickets.append(S.submit_cg(ids["f64"][i], bs[i], xs[j], rtol=1e-10, max_iter=500))
            else:
                low = "bf16" if mode == "refine_bf16" else "f32"
                tickets.append(S.submit_cg_refine(ids["f64"][i], ids[low][i], bs[i], xs[j], rtol=1e-10, max_iter=500))
        resp = [S.wait(t) for t in tickets]
        st = S.stats()
        S.close()
        true_res = [solvers.residual(csrs[pick[j]], bs[pick[j]], xs[j]) for j in check]
        out[mode] = {"solves_per_s": st["solves_per_s"], "p50_ms": st["p50_us"] / 1e3, "p99_ms": st["p99_us"] / 1e3,
                     "converged": sum(1 for r in resp if r["converged"]),
                     "mean_iterations": float(np.mean([r["iterations"] for r in resp])),
                     "replacements": int(sum(r["replacements"] for r in resp)),
                     "max_true_residual_oracle": float(max(true_res)), "oracle_checked": len(check)}
        log(f"serving precision, {mode}: {json.dumps(out[mode])}")
    for vt in H:
        for M in H[vt]:
            M.close()
    base = out["fp64_cg"]["solves_per_s"]
    out["speedup_vs_fp64"] = {m: out[m]["solves_per_s"] / base for m in ("fp64_cg", "refine_bf16", "refine_f32")}
    return out


SERVE_WORKLOAD = ("serving: 256 resident matrices (3D block, power-law, 3D Poisson; n log-uniform in [1e3, 1e6]; "
                  "FP64 and FP32), SpMM k in 1..16 or CG requests to 1e-10 (cap 500; FP32 matrices: FP64 "
                  "residual replacement)")


def run_serve(args, cb, matgen) -> int:
    r = serve_legs(args, cb, matgen, args.requests)
    st_b = r["all_at_once"]
    out = {
        "metric": "batched solves/s, p50/p99 (serving)",
        "value": round(st_b["solves_per_s"], 2), "unit": "solves/s", "n_gpus": 1, "steps": r["requests"],
        "warmup": 1, "ms_per_step": 1e3 / st_b["requests_per_s"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": SERVE_WORKLOAD, "requests": r["requests"], "cg_requests": r["cg_requests"]},
        "roofline": None, "cpu_baseline": None,
        "extra": {k: v for k, v in r.items() if k not in ("requests", "cg_requests")},
    }
    print(json.dumps(out), flush=True)
    return 0


def run_ablation(args, cb, matgen) -> int:
    """Section 4's ablation (Fig. 12) on the synthetic matrices, FP64: SpMV time under each option
    set of diagnostics.ABLATION; the non-zeros-per-tile histogram of the plain partition (Fig. 3);
    non-zeros per unit of work with and without Algorithm 2 (Fig. 4); converter time against nnz
    (Fig. 13(b)) on the block matrix at three sizes."""
    import torch

    from paper_2605_18515_amd import diagnostics

    res = {}
    for wl in ("block3d", "poisson", "powerlaw"):
        A = make_matrix(wl, 100)
        x = torch.from_numpy(matgen.vector(A.n, 1)).to("cuda")
        y = torch.empty(A.m, dtype=torch.float64, device="cuda")
        row = {"nnz": A.nnz}
        for name, opts in diagnostics.ABLATION.items():
            M = cb.CbMatrix.from_csr(A, **opts)
            settle(lambda: M.spmv(x, y), 0.3)
            _, k = time_calls(lambda: M.spmv(x, y), 100, 10)
            inf = M.info
            row[name] = {"us": k * 1e6, "gflops": 2.0 * A.nnz / k / 1e9, "spmv_bytes": inf["spmv_bytes"],
                         "convert_seconds": inf["convert_seconds"], "col_agg": inf["col_agg"],
                         "tiles": inf["ntiles"], "balance": diagnostics.balance(M)}
            if name == "CB-I":
                row["tile_histogram_plain"] = diagnostics.tile_nnz_histogram(M)
            M.close()
            log(f"{wl} {name}: {k * 1e6:.1f} us, {2.0 * A.nnz / k / 1e9:.0f} GFLOP/s, tiles {inf['ntiles']}, "
                f"wave nnz std {row[name]['balance']['wave_nnz_std']:.0f}, "
                f"quantum nnz std {row[name]['balance']['quantum_nnz_std']:.0f}")
        base = row["CB-I"]["us"]
        row["speedup_vs_CB-I"] = {n: base / row[n]["us"] for n in diagnostics.ABLATION}
        log(f"{wl}: speedup over CB-I {row['speedup_vs_CB-I']}; plain tiles by nnz "
            f"{row['tile_histogram_plain']['shares']}")
        res[wl] = row
        del x, y
        torch.cuda.empty_cache()
    conv = []
    for side in (25, 50, 100):
        A = matgen.block_3d(side, 3, 10.0, seed=1)
        M = cb.CbMatrix.from_csr(A, device=False)
        conv.append({"nnz": A.nnz, "convert_seconds": M.info["convert_seconds"]})
        M.close()
    log(f"converter time against nnz: {conv}")
    out = {"metric": "ablation: SpMV speedup of the full method over CB-I (3D block matrix, FP64)",
           "value": round(res["block3d"]["speedup_vs_CB-I"]["CB (contiguous)"], 4), "unit": "x", "n_gpus": 1,
           "steps": 100, "warmup": 10, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "ablation on the 3D block (100^3 x 3), 192^3 Poisson and 4M power-law matrices"},
           "roofline": None, "cpu_baseline": None, "extra": {"matrices": res, "converter": conv}}
    print(json.dumps(out), flush=True)
    return 0


def run_tune(args, cb, matgen) -> int:
    """cb_tune on the three full-size matrices in FP64 and FP32 storage: SpMV time with the default
    options against the tuned ones (HIP events, 100 launches each), and the tuner's own time."""
    import numpy as np
    import torch

    rows = {}
    for wl in ("block3d", "poisson", "powerlaw"):
        A = make_matrix(wl, 100)
        x = matgen.vector(A.n, 1)
        for vt in ("f64", "f32"):
            dt = torch.float64 if vt == "f64" else torch.float32
            xd = torch.from_numpy(x).to("cuda", dt)
            yd = torch.empty(A.m, dtype=dt, device="cuda")
            M = cb.CbMatrix.from_csr(A, value_type=vt)
            settle(lambda: M.spmv(xd, yd), 0.3)
            _, k_def = time_calls(lambda: M.spmv(xd, yd), 100, 10)
            M.close()
            t = time.perf_counter()
            Mt, best, cands = cb.cb_tune(A, value_type=vt)
            tune_s = time.perf_counter() - t
            settle(lambda: Mt.spmv(xd, yd), 0.3)
            _, k_tun = time_calls(lambda: Mt.spmv(xd, yd), 100, 10)
            it = Mt.info
            Mt.close()
            key = f"{wl}_{vt}"

            def desc(c):
                o = c["opt"]
                return {"tile_dim": c["tile_dim"], "spmv_kernel": c["spmv_kernel"], "col_agg": c["col_agg"],
                        "th1": o["th1"], "th2": o["th2"], "row_reduce": c["row_reduce"], "lb_mode": o["lb_mode"],
                        "wave_nnz": o["wave_nnz"], "xcd_chunk": o["xcd_chunk"], "cols16": o["cols16"], "us": c["us"]}
            rows[key] = {"default_us": k_def * 1e6, "tuned_us": k_tun * 1e6, "speedup": k_def / k_tun,
                         "tune_seconds": tune_s, "candidates": [desc(c) for c in cands],
                         "best": {k: best[k] for k in ("col_agg", "th1", "th2", "row_reduce", "lb_mode", "wave_nnz",
                                                       "xcd_chunk", "tile_dim", "spmv_kernel", "cols16")},
                         "tuned_structure": {k: it[k] for k in ("tile_dim", "spmv_kernel", "col_agg", "row_reduce",
                                                                "xcd_chunk", "cols16", "ntiles")}}
            log(f"{key}: default {k_def * 1e6:.1f} us, tuned {k_tun * 1e6:.1f} us ({k_def / k_tun:.3f}x) "
                f"in {tune_s:.1f}s, chosen {rows[key]['tuned_structure']}; candidates: " + "; ".join(
                    f"S={c['tile_dim']} k{c['spmv_kernel']} agg={c['col_agg']} th=({c['opt']['th1']},{c['opt']['th2']}) "
                    f"rr={c['row_reduce']} lb={c['opt']['lb_mode']} wn={c['opt']['wave_nnz']} "
                    f"xcd={c['opt']['xcd_chunk']} c16={c['opt']['cols16']} {c['us']:.1f}" for c in cands))
            del xd, yd
            torch.cuda.empty_cache()
    geo = float(np.exp(np.mean([np.log(r["speedup"]) for r in rows.values()])))
    out = {"metric": "autotuned SpMV speedup over default options (geometric mean)", "value": round(geo, 4),
           "unit": "x", "n_gpus": 1, "steps": 100, "warmup": 10, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
           "config": {"workload": "cb_tune on the 3D block (100^3 x 3), 192^3 Poisson and 4M power-law matrices"},
           "roofline": None, "cpu_baseline": None, "extra": rows}
    print(json.dumps(out), flush=True)
    return 0


def run_tune_spmm(args, cb, matgen) -> int:
    """cb_tune with k right-hand sides on the FP32 and BF16 copies of the 3D block matrix: SpMM time
    with the default options against the tuned ones (HIP events, 20 launches each after a settle)."""
    import torch

    k = args.tune_spmm
    A = make_matrix("block3d", 100)
    Xd = torch.from_numpy(matgen.rhs_columns(A.n, k, 3)).to("cuda", torch.float32)
    Yd = torch.empty((A.m, k), dtype=torch.float32, device="cuda")
    rows = {}
    for vt in ("f32", "bf16"):
        M = cb.CbMatrix.from_csr(A, value_type=vt)
        settle(lambda: M.spmm(Xd, Yd), 0.3)
        _, k_def = time_calls(lambda: M.spmm(Xd, Yd), 20, 2)
        M.close()
        t = time.perf_counter()
        Mt, best, cands = cb.cb_tune(A, value_type=vt, spmm_k=k)
        tune_s = time.perf_counter() - t
        settle(lambda: Mt.spmm(Xd, Yd), 0.3)
        _, k_tun = time_calls(lambda: Mt.spmm(Xd, Yd), 20, 2)
        it = Mt.info
        Mt.close()
        rows[vt] = {"default_us": k_def * 1e6, "tuned_us": k_tun * 1e6, "speedup": k_def / k_tun,
                    "tune_seconds": tune_s,
                    "tuned_structure": {n: it[n] for n in ("tile_dim", "col_agg", "xcd_chunk", "nwaves", "ntiles")},
                    "best": {n: best[n] for n in ("col_agg", "th1", "th2", "lb_mode", "wave_nnz", "xcd_chunk",
                                                  "tile_dim")},
                    "candidates": [{"us": c["us"], "tile_dim": c["tile_dim"], "col_agg": c["col_agg"],
                                    "wave_nnz": c["opt"]["wave_nnz"], "xcd_chunk": c["opt"]["xcd_chunk"],
                                    "lb_mode": c["opt"]["lb_mode"], "th": [c["opt"]["th1"], c["opt"]["th2"]]}
                                   for c in cands]}
        log(f"spmm k={k} {vt}: default {k_def * 1e6:.1f} us, tuned {k_tun * 1e6:.1f} us "
            f"({k_def / k_tun:.3f}x) in {tune_s:.1f}s, chosen {rows[vt]['tuned_structure']} {rows[vt]['best']}")
    out = {"metric": f"autotuned SpMM (k = {k}) speedup over default options", "value": None, "unit": "x",
           "n_gpus": 1, "steps": 20, "warmup": 2, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+bf16", "data": "synthetic",
           "config": {"workload": f"cb_tune with {k} right-hand sides on the 3D block matrix (100^3 x 3)"},
           "roofline": None, "cpu_baseline": None, "extra": rows}
    out["value"] = round(min(r["speedup"] for r in rows.values()), 4)
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--side", type=int, default=100, help="grid side of the 3D block matrix")
    ap.add_argument("--workload", default="block3d", choices=list(WORKLOADS),
                    help="matrix: block3d (default, 100^3 x 3 dof), powerlaw (n = 4M, Zipf 2.1 rows, mean 16), "
                         "powerlaw_literal (the same rows unscaled, mean 4.8), "
                         "poisson (7-point, 192^3), laplacian (5-point, 64 x 64)")
    ap.add_argument("--lb", default="contiguous", choices=["contiguous", "paper", "none", "paper_stream"])
    ap.add_argument("--col-agg", type=int, default=-1)
    ap.add_argument("--wave-nnz", type=int, default=0)
    ap.add_argument("--spmv-kernel", type=int, default=-1,
                    help="natural-order SpMV kernel of the handles (cb_options_t.spmv_kernel; -1 the library's "
                         "default)")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP32/BF16, SpMM and copy legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle check of the result")
    ap.add_argument("--no-solves", action="store_true",
                    help="skip the CG (FP64 vs mixed) and serving legs of the extra measurements")
    ap.add_argument("--serve-requests", type=int, default=500, help="requests of the serving leg of the extras")
    ap.add_argument("--serve-active", type=int, default=128, help="solve slots per vector type of the server")
    ap.add_argument("--serve-tune", action="store_true",
                    help="serving workload: handles take cb_tune's options per matrix family and value type")
    ap.add_argument("--serve-min-wave-nnz", type=int, default=1024,
                    help="min_wave_nnz of the serving workload's handles (0: the library's automatic floor)")
    ap.add_argument("--serve-arena-gib", type=int, default=16, help="device arena of the server, GiB")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--settle-seconds", type=float, default=1.0,
                    help="untimed launches of the headline SpMV for this long after the warm-up, before the "
                         "timed region (clocks reach their steady state); reported in extra.untimed_settle")
    ap.add_argument("--leg-settle-seconds", type=float, default=0.3,
                    help="the same before each leg of the extra measurements")
    ap.add_argument("--graph", action="store_true",
                    help="time the SpMV steps as replays of one captured HIP graph (launch-bound workloads)")
    ap.add_argument("--cg", action="store_true",
                    help="instead of the SpMV line: CG solves/s on the 192^3 Poisson operator to a true FP64 "
                         "residual of 1e-10, FP64 CG against the mixed-precision solvers on FP32 and BF16 copies")
    ap.add_argument("--serve", action="store_true",
                    help="instead of the SpMV line: the serving workload (256 resident matrices, SpMM and CG "
                         "requests with Poisson arrivals), p50/p99 latency and solves/s")
    ap.add_argument("--requests", type=int, default=1000, help="requests of the serving workload")
    ap.add_argument("--ablation", action="store_true",
                    help="instead of the SpMV line: the ablation (CB-I, CB-II, full with Algorithm 2 and with the "
                         "contiguous split) on the three full-size matrices in FP64, the tile histogram, the work "
                         "balance and the converter's time against nnz")
    ap.add_argument("--tune", action="store_true",
                    help="instead of the SpMV line: the autotuner on the block, Poisson and power-law matrices in "
                         "FP64 and FP32, tuned against default options")
    ap.add_argument("--tune-spmm", type=int, default=0, metavar="K",
                    help="instead of the SpMV line: the autotuner timing SpMM with K right-hand sides on the "
                         "FP32 and BF16 block matrix, tuned against default options")
    ap.add_argument("--copy-only", type=int, default=0, metavar="MIB",
                    help="only run the streaming copy kernel over MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the CB-SpMV path here runs on a single MI355X "
              "(no multi-GPU sharding is implemented); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2605_18515_amd import matgen
    from paper_2605_18515_amd import cbspmv as cb

    # the stencil and power-law legs of the extras need their matrices; worker processes (forked
    # before this process touches the GPU, CPU work only) generate them while this process
    # generates and converts the block matrix
    pool, pending = None, {}
    if (not args.no_extras and args.workload == "block3d" and not args.copy_only and not args.cg and not args.serve
            and not args.tune and not args.tune_spmm and not args.ablation):
        import multiprocessing as mp

        pool = mp.get_context("fork").Pool(2)
        pending = {wl: pool.apply_async(make_matrix, (wl, 0)) for wl in ("powerlaw", "poisson")}

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.copy_only:
        nbytes = args.copy_only << 20
        src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        w_s, k_s = time_calls(lambda: cb.cb_copy_probe(src, dst, nbytes), args.steps, args.warmup)
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": args.steps + args.warmup,
                          "GBs": 2 * nbytes / k_s / 1e9}), flush=True)
        return 0
    if args.cg:
        return run_cg(args, cb, matgen)
    if args.serve:
        return run_serve(args, cb, matgen)
    if args.tune:
        return run_tune(args, cb, matgen)
    if args.tune_spmm:
        return run_tune_spmm(args, cb, matgen)
    if args.ablation:
        return run_ablation(args, cb, matgen)
    t = time.perf_counter()
    A = make_matrix(args.workload, args.side)
    x = matgen.vector(A.n, 1)
    log(f"generated {args.workload} matrix n={A.n} nnz={A.nnz} in {time.perf_counter() - t:.1f}s")

    t = time.perf_counter()
    M = cb.CbMatrix.from_csr(A, lb_mode=args.lb, col_agg=args.col_agg, wave_nnz=args.wave_nnz,
                             spmv_kernel=args.spmv_kernel)
    create_s = time.perf_counter() - t
    info = M.info
    log(f"converted+uploaded in {create_s:.2f}s (convert {info['convert_seconds']:.2f}s): {info['ntiles']} tiles "
        f"coo/csr/dense {info['tiles_coo']}/{info['tiles_csr']}/{info['tiles_dense']} col_agg={info['col_agg']} "
        f"waves={info['nwaves']} shared={info['shared_panels']} bytes={info['spmv_bytes']}")

    xd = torch.from_numpy(x).to(dev)
    yd = torch.empty(A.m, dtype=torch.float64, device=dev)
    step = lambda: M.spmv(xd, yd)  # noqa: E731
    # the background generation ends before any timed region: host processes competing with the
    # launching thread leave the GPU idle between short kernels (the BF16 leg read 83-91 us instead
    # of 77 while they ran)
    ready = {wl: r.get() for wl, r in pending.items()}
    if pool is not None:
        pool.close()
        pool.join()
        pool = None
    sclk0 = gpu_sclk()
    for _ in range(args.warmup):
        step()
    settled = settle(step, args.settle_seconds) if not args.graph else None
    wall_s, kern_s = (time_graph if args.graph else time_calls)(step, args.steps, 0)
    sclk1 = gpu_sclk()
    gflops = 2.0 * A.nnz / wall_s / 1e9
    achieved = info["spmv_bytes"] / kern_s / 1e9
    log(f"FP64 SpMV: {wall_s * 1e6:.1f} us/step wall, {kern_s * 1e6:.1f} us kernel, {gflops:.1f} GFLOP/s, "
        f"{achieved:.0f} GB/s algorithmic (clock before warm-up {sclk0}, after the timed launches {sclk1})")

    err = None
    coo = None
    if not args.no_check or not args.no_cpu:
        import oracle

        coo = (np.repeat(np.arange(A.m, dtype=np.int32), np.diff(A.row_ptr)), A.col_idx, A.values)
    if not args.no_check:
        y = yd.cpu().numpy()
        ref = oracle.spmv(A, x, comp=True, coo=coo)
        err, viol, _ = oracle.scaled_error(y, ref, oracle.scale(A, x, coo=coo), 1e-12)
        log(f"oracle check: max scaled error {err:.3e}, violations {viol}")
        if viol:
            log("FAILED: result outside the 1e-12 tolerance")
            return 1

    # the paper's width model of the same structure (21 bytes of metadata per tile, payload, column maps)
    paper_bytes = info["meta_bytes"] + info["payload_bytes"] + info["restore_bytes"] + 8 * (A.n + A.m)
    extra = {"bytes_paper_model": paper_bytes, "GBs_paper_model": paper_bytes / kern_s / 1e9,
             "convert_seconds": info["convert_seconds"], "create_seconds": create_s,
             "kernel_us": kern_s * 1e6, "max_scaled_error_fp64": err,
             "untimed_settle": None if settled is None else
             {"launches": settled[0], "seconds": settled[1],
              "note": "untimed launches after the warm-up and before the timed region, until the GPU's "
                      "clocks reach the steady state of a long run"},
             "sclk": {"before_warmup": sclk0, "after_timed": sclk1},
             "structure": {k: info[k] for k in ("ntiles", "tiles_coo", "tiles_csr", "tiles_dense", "col_agg",
                                                "super_sparse_share", "payload_bytes", "meta_bytes",
                                                "restore_bytes", "sched_bytes", "nwaves", "shared_panels",
                                                "wave_nnz_max", "wave_nnz_mean", "spmv_bytes")}}

    if not args.no_extras:
        # achievable bandwidth of a plain streaming copy on this device
        nbytes = 1 << 30
        src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        cw, ck = time_calls(lambda: cb.cb_copy_probe(src, dst, nbytes), 20, 3)
        extra["copy_probe_GBs"] = 2 * nbytes / ck / 1e9
        # and of a read-only stream (the product reads its structure and x and writes only y)
        sink = torch.zeros(2, dtype=torch.float64, device=dev)
        rw, rk = time_calls(lambda: cb.cb_read_probe(src, nbytes, sink), 20, 3)
        extra["read_probe_GBs"] = nbytes / rk / 1e9
        extra["spmv_frac_of_read_probe"] = achieved / extra["read_probe_GBs"]
        del src, dst, sink
        log(f"copy probe: {extra['copy_probe_GBs']:.0f} GB/s; read probe: {extra['read_probe_GBs']:.0f} GB/s "
            f"(the product's algorithmic rate is {100 * extra['spmv_frac_of_read_probe']:.1f} % of it)")
        M.close()
        torch.cuda.empty_cache()
        import oracle

        lsteps = max(50, args.steps // 3)
        srows = sample_rows(A, 4096, 7)
        sub = rows_of(A, srows)
        for vt in ("f32", "bf16"):
            Mv = cb.CbMatrix.from_csr(A, value_type=vt, lb_mode=args.lb, col_agg=args.col_agg,
                                      wave_nnz=args.wave_nnz, spmv_kernel=args.spmv_kernel)
            iv = Mv.info
            x32 = torch.from_numpy(x).to(dev, torch.float32)
            y32 = torch.empty(A.m, dtype=torch.float32, device=dev)
            spmv32 = lambda: Mv.spmv(x32, y32)  # noqa: E731
            settle(spmv32, args.leg_settle_seconds)
            w1, k1 = time_calls(spmv32, lsteps, 0)
            leg = {"spmv_gflops": 2.0 * A.nnz / w1 / 1e9, "spmv_kernel_us": k1 * 1e6,
                   "spmv_GBs": iv["spmv_bytes"] / k1 / 1e9, "spmv_frac": iv["spmv_bytes"] / k1 / 1e9 / HBM_PEAK_GBS,
                   "spmv_bytes": iv["spmv_bytes"], "row_reduce": iv["row_reduce"]}
            if not args.no_check:
                e, _, _ = oracle.scaled_error(y32.cpu().double().numpy(), ref, oracle.scale(A, x, coo=coo), 1.0)
                leg["max_scaled_error_vs_fp64_oracle"] = e
            del x32, y32
            for k in (8, 32):
                # X column j from seed 3 + j, rounded to FP32; checked on sampled rows against the FP64
                # oracle on the original values and X
                Xh = matgen.rhs_columns(A.n, k, 3)
                Xd = torch.from_numpy(Xh).to(dev, torch.float32)
                Yd = torch.empty((A.m, k), dtype=torch.float32, device=dev)
                spmmk = lambda: Mv.spmm(Xd, Yd)  # noqa: E731
                settle(spmmk, args.leg_settle_seconds)
                wk, kk = time_calls(spmmk, 20, 0)
                # the SpMV structure's bytes with X and Y in place of x and y; the SpMM kernel reads the
                # tiles' 4-byte original columns, not the SpMV kernels' 2-byte offsets
                S_ = iv["tile_dim"]
                c16 = {0: 0, 1: 2 * S_ - 4, 2: 2 * S_}[iv["cols16"]] * iv["ntiles"]
                sb = iv["spmv_bytes"] + c16 - 4 * (A.n + A.m) + 4 * k * (A.n + A.m)
                leg[f"spmm_k{k}_gflops"] = 2.0 * A.nnz * k / wk / 1e9
                leg[f"spmm_k{k}_kernel_us"] = kk * 1e6
                leg[f"spmm_k{k}_bytes"] = sb
                leg[f"spmm_k{k}_GBs"] = sb / kk / 1e9
                if not args.no_check:
                    Ys = Yd.cpu().double().numpy()[srows]
                    refk = oracle.spmm(sub, Xh)
                    sclk = oracle.spmm(matgen.Csr(sub.m, sub.n, sub.row_ptr, sub.col_idx, np.abs(sub.values)),
                                       np.abs(Xh))
                    ek, vk, _ = oracle.scaled_error(Ys.ravel(), refk.ravel(), sclk.ravel(), STORAGE_TOL[vt])
                    leg[f"spmm_k{k}_max_scaled_error_vs_fp64_oracle"] = ek
                    leg[f"spmm_k{k}_checked_rows"] = int(srows.size)
                    if vk:
                        log(f"FAILED: {vt} SpMM k={k} outside {STORAGE_TOL[vt]} on sampled rows (max {ek:.3e})")
                        return 1
                del Xd, Yd, Xh
            extra[vt] = leg
            log(f"{vt}: {json.dumps(leg)}")
            Mv.close()
            torch.cuda.empty_cache()
        ref = sub = None  # (ref is only computed when results are checked)
        # the other FP64 workloads of the metric, each checked row by row against the oracle: the
        # stencil family at scale (192^3 Poisson), the power-law rows, and the 64 x 64 Laplacian,
        # whose whole working set sits in cache (launch latency, not HBM)
        for wl in ("poisson", "powerlaw"):
            Aw = ready.pop(wl) if wl in ready else make_matrix(wl, 0)
            extra[f"spmv_{wl}"] = spmv_leg(cb, Aw, dev, lsteps, args.leg_settle_seconds, not args.no_check,
                                           WORKLOADS[wl], spmv_kernel=args.spmv_kernel)
            log(f"{wl}: {json.dumps(extra[f'spmv_{wl}'])}")
            del Aw
            torch.cuda.empty_cache()
        extra["laplacian64"] = laplacian_leg(cb, dev, not args.no_check)
        log(f"laplacian 64x64: {json.dumps(extra['laplacian64'])}")
        if not args.no_solves:
            # the metric's other half: solves/s of FP64 CG against the mixed-precision solver, and of the
            # serving loop's batches against one request at a time, with p50/p99 latency
            legs, _, ok = cg_legs(args, cb, matgen, ("fp64_cg", "replace_f32", "replace_bf16"))
            base = legs["fp64_cg"]["solves_per_s"]
            extra["cg_poisson192"] = {
                k: {kk: v[kk] for kk in ("solves_per_s", "iterations", "refinements", "rel_residual_oracle")
                    if kk in v} for k, v in legs.items()}
            extra["cg_poisson192"]["speedup_vs_fp64_cg"] = {k: v["solves_per_s"] / base for k, v in legs.items()}
            if not ok:
                log("FAILED: a CG solve missed the 1e-10 residual")
                return 1
            srv = serve_legs(args, cb, matgen, args.serve_requests)
            extra["serving"] = {
                "workload": SERVE_WORKLOAD, "requests": srv["requests"], "cg_requests": srv["cg_requests"],
                "batched_solves_per_s": srv["all_at_once"]["solves_per_s"],
                "one_at_a_time_solves_per_s": srv["one_at_a_time"]["solves_per_s"],
                "speedup_solves": srv["speedup_solves_vs_one_at_a_time"],
                "poisson_arrivals_per_s": srv["poisson_arrivals"]["rate_per_s"],
                "p50_ms": srv["poisson_arrivals"]["p50_us"] / 1e3, "p99_ms": srv["poisson_arrivals"]["p99_us"] / 1e3,
                "arrival_sweep": srv["arrival_sweep"],
                "cg_converged": srv["cg_converged"], "refined_requests": srv["refined_requests"], "rtol": srv["rtol"],
                "max_rel_diff_vs_one_at_a_time": srv["max_rel_diff_vs_one_at_a_time"],
                "precision": srv["precision"]}
    else:
        M.close()

    cpu = None
    if not args.no_cpu:
        import oracle

        w = np.empty(A.m)
        lib = oracle.lib()
        rows, cols, vals = coo
        yb = np.empty(A.m)
        reps, t0 = 0, time.perf_counter()
        while True:
            lib.oracle_spmv_coo(A.m, A.nnz, rows.ctypes.data, cols.ctypes.data, vals.ctypes.data, x.ctypes.data,
                                1.0, 0.0, None, yb.ctypes.data, w.ctypes.data)
            reps += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        cpu = {"value": 2.0 * A.nnz * reps / el / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
               "sample": f"the full {args.workload} matrix ({A.nnz} nnz), {reps} plain FP64 COO-loop SpMVs in "
                         f"{el:.1f}s on one host core"}
        log(f"cpu oracle: {cpu['value']:.3f} GFLOP/s")
        # the same rows on every core this process may use (a CSR loop, not the oracle's COO loop)
        ncores = len(os.sched_getaffinity(0))
        rp, ci, va = (np.ascontiguousarray(A.row_ptr), np.ascontiguousarray(A.col_idx),
                      np.ascontiguousarray(A.values))
        reps, t0 = 0, time.perf_counter()
        while True:
            lib.oracle_spmv_csr_par(A.m, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, x.ctypes.data, 1.0,
                                    yb.ctypes.data, ncores)
            reps += 1
            if time.perf_counter() - t0 >= min(3.0, args.cpu_seconds):
                break
        el = time.perf_counter() - t0
        extra["cpu_all_cores"] = {"value": 2.0 * A.nnz * reps / el / 1e9, "unit": "GFLOP/s", "cores": ncores,
                                  "sample": f"{reps} CSR-loop SpMVs on {ncores} threads in {el:.1f}s"}
        log(f"cpu all cores ({ncores}): {extra['cpu_all_cores']['value']:.2f} GFLOP/s")

    traffic = measured_traffic(A.nnz, info["spmv_bytes"])
    out = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload].format(side=args.side), "n": A.n, "nnz": A.nnz,
                   "lb_mode": args.lb, "timing": "hip graph replay" if args.graph else "stream launches",
                   "col_agg": info["col_agg"], "value_storage": "f64"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": info["spmv_bytes"], "kernel": kernel_name(info, args.lb)},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    return 0

if __name__ == "__main__":
    sys.exit(main())
