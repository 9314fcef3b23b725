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
    "poisson": "FP64 y=A*x, 3D 7-point Poisson operator on a 192^3 grid",
    "laplacian": "FP64 y=A*x, 2D 5-point Laplacian on a 64x64 grid",
}


def make_matrix(name: str, side: int):
    from paper_2605_18515_amd import matgen

    if name == "block3d":
        return matgen.block_3d(side, 3, 10.0, seed=1)
    if name == "powerlaw":
        return matgen.power_law(4_000_000, seed=2)
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


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, when
    they were taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
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


def run_cg(args, cb, matgen) -> int:
    """Solves of A x = b from x = 0 on the 192^3 Poisson operator (b ~ U[-1, 1]) until the FP64
    residual |b - A x| / |b| is at most 1e-10: FP64 CG, and the two mixed-precision solvers
    (residual replacement and restarted refinement) with the products on the FP32 and on the BF16
    copy of A.  Each solve is timed whole (host polling included)."""
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
    for name in ("fp64_cg", "replace_f32", "replace_bf16", "replace_f32w", "replace_bf16w", "restart_f32",
                 "restart_bf16", "restart_f32w"):
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
    best = max(legs, key=lambda k: legs[k]["solves_per_s"])
    out = {
        "metric": "CG solves/s to |b - Ax| / |b| <= 1e-10 (FP64 vs mixed-precision refinement)",
        "value": round(legs[best]["solves_per_s"], 4), "unit": "solves/s", "n_gpus": 1,
        "steps": len(times), "warmup": 1, "ms_per_step": legs[best]["seconds"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "CG on the 3D 7-point Poisson operator, 192^3 grid, b ~ U[-1,1], x0 = 0",
                   "n": A.n, "nnz": A.nnz, "method": best},
        "roofline": None, "cpu_baseline": None,
        "extra": {"legs": legs, "speedup_vs_fp64_cg": {k: legs[k]["solves_per_s"] / legs["fp64_cg"]["solves_per_s"]
                                                       for k in legs}},
    }
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--side", type=int, default=100, help="grid side of the 3D block matrix")
    ap.add_argument("--workload", default="block3d", choices=list(WORKLOADS),
                    help="matrix: block3d (default, 100^3 x 3 dof), powerlaw (n = 4M, Zipf 2.1 rows, mean 16), "
                         "poisson (7-point, 192^3), laplacian (5-point, 64 x 64)")
    ap.add_argument("--lb", default="contiguous", choices=["contiguous", "paper", "none"])
    ap.add_argument("--col-agg", type=int, default=-1)
    ap.add_argument("--wave-nnz", type=int, default=0)
    ap.add_argument("--no-extras", action="store_true", help="skip the FP32/BF16, SpMM and copy legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle check of the result")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--graph", action="store_true",
                    help="time the SpMV steps as replays of one captured HIP graph (launch-bound workloads)")
    ap.add_argument("--cg", action="store_true",
                    help="instead of the SpMV line: CG solves/s on the 192^3 Poisson operator to a true FP64 "
                         "residual of 1e-10, FP64 CG against the mixed-precision solvers on FP32 and BF16 copies")
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
    t = time.perf_counter()
    A = make_matrix(args.workload, args.side)
    x = matgen.vector(A.n, 1)
    log(f"generated {args.workload} matrix n={A.n} nnz={A.nnz} in {time.perf_counter() - t:.1f}s")

    t = time.perf_counter()
    M = cb.CbMatrix.from_csr(A, lb_mode=args.lb, col_agg=args.col_agg, wave_nnz=args.wave_nnz)
    create_s = time.perf_counter() - t
    info = M.info
    log(f"converted+uploaded in {create_s:.2f}s (convert {info['convert_seconds']:.2f}s): {info['ntiles']} tiles "
        f"coo/csr/dense {info['tiles_coo']}/{info['tiles_csr']}/{info['tiles_dense']} col_agg={info['col_agg']} "
        f"waves={info['nwaves']} shared={info['shared_panels']} bytes={info['spmv_bytes']}")

    xd = torch.from_numpy(x).to(dev)
    yd = torch.empty(A.m, dtype=torch.float64, device=dev)
    step = lambda: M.spmv(xd, yd)  # noqa: E731
    wall_s, kern_s = (time_graph if args.graph else time_calls)(step, args.steps, args.warmup)
    gflops = 2.0 * A.nnz / wall_s / 1e9
    achieved = info["spmv_bytes"] / kern_s / 1e9
    log(f"FP64 SpMV: {wall_s * 1e6:.1f} us/step wall, {kern_s * 1e6:.1f} us kernel, {gflops:.1f} GFLOP/s, "
        f"{achieved:.0f} GB/s algorithmic")

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

    extra = {"convert_seconds": info["convert_seconds"], "create_seconds": create_s,
             "kernel_us": kern_s * 1e6, "max_scaled_error_fp64": err,
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
        del src, dst
        log(f"copy probe: {extra['copy_probe_GBs']:.0f} GB/s")
        M.close()
        torch.cuda.empty_cache()
        import oracle

        for vt in ("f32", "bf16"):
            Mv = cb.CbMatrix.from_csr(A, value_type=vt, lb_mode=args.lb, col_agg=args.col_agg,
                                      wave_nnz=args.wave_nnz)
            iv = Mv.info
            x32 = torch.from_numpy(x).to(dev, torch.float32)
            y32 = torch.empty(A.m, dtype=torch.float32, device=dev)
            w1, k1 = time_calls(lambda: Mv.spmv(x32, y32), max(50, args.steps // 3), 5)
            leg = {"spmv_gflops": 2.0 * A.nnz / w1 / 1e9, "spmv_kernel_us": k1 * 1e6,
                   "spmv_GBs": iv["spmv_bytes"] / k1 / 1e9, "spmv_bytes": iv["spmv_bytes"]}
            if not args.no_check:
                e, _, _ = oracle.scaled_error(y32.cpu().double().numpy(), ref, oracle.scale(A, x, coo=coo), 1.0)
                leg["max_scaled_error_vs_fp64_oracle"] = e
            for k in (8, 32):
                Xd = torch.empty((A.n, k), dtype=torch.float32, device=dev).uniform_(-1, 1)
                Yd = torch.empty((A.m, k), dtype=torch.float32, device=dev)
                wk, kk = time_calls(lambda: Mv.spmm(Xd, Yd), 20, 3)
                leg[f"spmm_k{k}_gflops"] = 2.0 * A.nnz * k / wk / 1e9
                leg[f"spmm_k{k}_kernel_us"] = kk * 1e6
                del Xd, Yd
            extra[vt] = leg
            log(f"{vt}: {json.dumps(leg)}")
            Mv.close()
            del x32, y32
            torch.cuda.empty_cache()
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

    traffic = measured_traffic()
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
                     "bytes_per_launch": info["spmv_bytes"], "kernel": "spmv_kernel<0>"},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
