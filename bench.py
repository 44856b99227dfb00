"""Benchmark of the MI355X AAR solver: solves/s at 1e-10 relative residual.

A step is one complete AAR solve (every stage of the iteration: fused
Richardson sweeps, Anderson residual and Gram reduction, pseudoinverse
solve, update; plus FP64 refinement in mixed mode) of one seeded synthetic
system whose right-hand side and solver workspace are already resident in
HBM.  Default workload: periodic Poisson, 192^3 grid, 12th-order central
differences (37-point stencil), 64 Gaussian charges minus their mean,
Jacobi preconditioner, omega = beta = 0.6, m = 7, p = 6, tol 1e-10, FP64.
The same grid is also solved in mixed precision (FP32 iteration inside FP64
refinement) and as FP64 with an FP32 history ring, each reported beside it
with the speedup over FP64, and the batched workload (512 shifted Helmholtz
systems in one call) runs in FP64 and mixed precision.

Prints one JSON line.  `roofline` covers the dominant kernel (the fused
Richardson sweep): algorithmic bytes per launch (read x and b, write x and
f: 4 values per grid point) over the mean launch time measured with HIP
events on the solver's stream, against the 8 TB/s HBM peak and against a
measured 1 GiB device copy.  `cpu_baseline` times the CPU oracle on a
bounded number of iterations of the same system and scales to solves/s with
the oracle's own iteration count.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "AAR solves/s and sweep HBM GB/s at 1e-10 rel-residual: mixed/batched vs FP64"
HBM_PEAK_GBS = 8000.0
# Oracle (FP64, CPU) iterations to 1e-10 on the default workload, written by
# tests/golden/make_golden.py (oracle only).
GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_full_size.json")
# HBM traffic of the sweep kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# scaled by a plain copy's counters; valid while the stencil sources and the
# grid's tile shape are those it was measured with.
SWEEP_PROFILE = os.path.join(ROOT, "profiles", "k_stencil2_sweep_fp64_r6_192.md")
STENCIL_SRCS = [os.path.join(ROOT, "paper_1606_08740_amd", "csrc", f)
                for f in ("stencil_kernels.h", "stencil.hip", "stencil_narrow.hip", "stencil_f32.hip")]


def stencil_sha():
    """First 16 hex digits of the SHA-256 of the stencil sources' code: the
    files concatenated with // comments, trailing blanks and empty lines
    removed, so editing a comment keeps a profile valid."""
    import hashlib
    h = hashlib.sha256()
    for f in STENCIL_SRCS:
        for line in open(f):
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def fp64_tile(n, radius=6):
    """The FP64 tile shape the library reads for an n^3 grid (the tile file
    named by AAR_TUNE_CACHE, else the one beside it), or None."""
    path = os.environ.get("AAR_TUNE_CACHE") or os.path.join(ROOT, "paper_1606_08740_amd", "tuned_tiles.txt")
    if not os.path.exists(path):
        return None
    tile = None
    for line in open(path):
        f = line.split()
        if len(f) >= 8 and not line.startswith("#") and f[:6] == ["0", str(radius), "0", str(n), str(n), str(n)]:
            v = [int(t) for t in f[6:10]] + [0] * (10 - len(f))
            tile = {"rows_per_thread": v[0], "z_depth": v[1], "order": v[2], "pair": v[3]}
    return tile


def sweep_traffic(n):
    """Counter-measured bytes per sweep launch, or None when absent or stale."""
    import re
    if n != 192 or not os.path.exists(SWEEP_PROFILE):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(SWEEP_PROFILE).read(), flags=re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("stencil_source_sha256_16") != stencil_sha() or rec.get("tile") != fp64_tile(n):
        return None
    return rec.get("traffic_bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=192)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=180)
    ap.add_argument("--kernel-timing-solves", type=int, default=1)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-count", type=int, default=512)
    ap.add_argument("--batched-steps", type=int, default=2)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scale for the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the batched part (for profiling it); prints its JSON object")
    ap.add_argument("--precision-only", choices=["mixed_fp32", "fp64_fp32hist"],
                    help="only time this precision mode on the headline system (for profiling it)")
    return ap.parse_args()


def measured_copy_gbs():
    """Device-to-device copy of 1 GiB of random doubles (no cache reuse between
    repetitions): the bandwidth a plain streaming kernel reaches on this GPU."""
    import torch
    src = torch.rand(1 << 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 5 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def copy_calibration():
    """A plain device-to-device copy of 2^27 doubles (1 GiB read, 1 GiB written),
    three times: the HBM counters of this kernel calibrate those of the solver."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8}))


def oracle_sample_error(x, n):
    """Max |x - x_oracle| over the 64 seeded sample points stored in the golden
    file (the oracle's FP64 solution of the same system, mean-free when the
    system is singular periodic), divided by the RMS of the oracle's solution;
    None when no stored solution exists for this size."""
    import numpy as np
    if not os.path.exists(GOLDEN):
        return None
    g = json.load(open(GOLDEN)).get(f"periodic_poisson_r6_{n}")
    if g is None:
        return None
    xs = x - x.mean() if g["mean_free"] else x
    rms = g["x_norm"] / np.sqrt(x.size)
    return float(np.max(np.abs(xs[g["sample_index"]] - np.asarray(g["sample_x"]))) / rms)


def timed_solves(solver, bt, steps, warmup):
    import torch
    res = None
    for _ in range(warmup):
        xt = torch.zeros_like(bt)
        res = solver.solve(bt, xt)
    xs = [torch.zeros_like(bt) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        res = solver.solve(bt, xs[i])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, res, xs[-1]


def run_batched(args):
    """The batched workload: 512 shifted periodic Helmholtz systems of uneven
    sizes solved by one aar_solve_batched call: FP64, mixed precision, and
    FP64 with an FP32 history ring."""
    import numpy as np
    import torch

    from paper_1606_08740_amd import aar, inputs
    wb = inputs.workload(5, count=args.batched_count)
    bb = torch.as_tensor(np.concatenate(wb.b), device="cuda:0")
    res_out = {"workload": f"{args.batched_count} periodic shifted Helmholtz systems, 8th-order "
                           "central FD (25-point), n ~ U{16..96}, sigma ~ U(0,10), b ~ N(0,1), "
                           "exact constant-mode deflation, tol 1e-10",
               "points": int(sum(p.size for p in wb.problems))}
    for label, prec in [("fp64", aar.AAR_FP64), ("mixed_fp32", aar.AAR_MIXED_FP32),
                        ("fp64_fp32hist", aar.AAR_FP64_FP32HIST)]:
        pb = inputs.Params(**{**wb.params.__dict__})
        pb.precision = prec
        sb = aar.Solver(wb.problems, pb)
        res = None
        for _ in range(max(args.warmup, 1)):
            xb = torch.zeros_like(bb)
            res = sb.solve_batched(bb, xb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batched_steps):
            xb = torch.zeros_like(bb)
            res = sb.solve_batched(bb, xb)
        torch.cuda.synchronize()
        dtb = (time.perf_counter() - t0) / args.batched_steps
        sb.close()
        its = [r["iterations"] for r in res]
        res_out[label] = {"value": args.batched_count / dtb, "unit": "solves/s",
                          "ms_per_call": dtb * 1e3,
                          "converged": int(sum(r["status"] == 0 for r in res)),
                          "iterations_total": int(sum(its)), "iterations_max": int(max(its)),
                          "max_rel_residual": float(max(r["rel_residual"] for r in res))}
    res_out["mixed_speedup_vs_fp64"] = res_out["mixed_fp32"]["value"] / res_out["fp64"]["value"]
    res_out["fp64_fp32hist_speedup_vs_fp64"] = res_out["fp64_fp32hist"]["value"] / res_out["fp64"]["value"]
    del bb
    return res_out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import numpy as np
    import torch

    from paper_1606_08740_amd import aar, inputs

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.batched_only:
        print(json.dumps(run_batched(args)))
        return
    w = inputs.workload(2, n=args.n)
    prob, b = w.problems[0], w.b[0]
    N = prob.size
    bt = torch.as_tensor(b, device="cuda:0")
    if args.precision_only:
        pm = w.params
        pm.precision = {"mixed_fp32": aar.AAR_MIXED_FP32, "fp64_fp32hist": aar.AAR_FP64_FP32HIST}[args.precision_only]
        sm = aar.Solver([prob], pm)
        dtm, rm, _ = timed_solves(sm, bt, args.steps, args.warmup)
        sm.close()
        print(json.dumps({"precision": args.precision_only, "value": args.steps / dtm, "unit": "solves/s",
                          "ms_per_step": dtm / args.steps * 1e3, "iterations": rm["iterations"],
                          "outer_steps": rm["outer_steps"], "rel_residual": rm["rel_residual"],
                          "status": rm["status"]}))
        return

    # ---- FP64 (headline) ----
    prm = w.params
    prm.precision = aar.AAR_FP64
    s64 = aar.Solver([prob], prm)
    dt64, r64, x64 = timed_solves(s64, bt, args.steps, args.warmup)
    # kernel timing pass: one HIP event pair around each cycle's p - 1 consecutive
    # sweep launches, on the solver's stream
    s64.set_timing(True)
    for _ in range(args.kernel_timing_solves):
        xt = torch.zeros_like(bt)
        s64.solve(bt, xt)
    ms_tot, launches = s64.sweep_time()
    s64.set_timing(False)
    s64.close()
    sweep_us = ms_tot / max(launches, 1) * 1e3
    # algorithmic bytes of the p - 1 Richardson sweeps of a cycle, per launch.
    # With the paired layout (and m + 1 >= p) the first sweep of a cycle reads
    # x and b and writes f (24 B per point); the others follow the residual
    # recursion f_{j+1} = f_j - omega D^-1 A f_j: read f_j, write f_{j+1}
    # (16 B).  Otherwise every sweep reads x, b and writes x, f (32 B).
    tile = fp64_tile(args.n)
    recursion = tile is not None and tile["pair"] > 0 and prm.m + 1 >= prm.p >= 2
    p = prm.p
    sweep_bytes = (3 * 8 + (p - 2) * 2 * 8) * N / (p - 1) if recursion else 4 * 8 * N
    achieved = sweep_bytes / (sweep_us * 1e-6) / 1e9

    out = {
        "metric": METRIC,
        "value": args.steps / dt64,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt64 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"periodic Poisson {args.n}^3, 12th-order central FD (37-point), "
                               "64 Gaussian charges minus mean, Jacobi, omega=beta=0.6, m=7, p=6, "
                               "tol 1e-10, FP64",
                   "grid": [args.n] * 3, "radius": 6, "m": 7, "p": 6, "tol": 1e-10, "precision": "fp64"},
        "iterations": r64["iterations"],
        "rel_residual": r64["rel_residual"],
        "status": r64["status"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": sweep_traffic(args.n),
                     "kernel": ("k_stencil2 Richardson sweeps, paired-point layout, FP64, radius 6: " +
                                ("a cycle's first from x and b, the others by the residual recursion"
                                 if recursion else "each from x and b")),
                     "bytes_per_launch": sweep_bytes, "mean_launch_us": sweep_us, "launches": launches},
    }
    xa = x64.cpu().numpy()
    out["error_vs_oracle"] = {
        "fp64": oracle_sample_error(xa, args.n),
        "measure": "max abs error at 64 seeded sample points over the RMS of the oracle's FP64 solution "
                   "(mean-free), stored in tests/golden/oracle_full_size.json by tests/golden/make_golden.py"}
    copy_gbs = measured_copy_gbs()
    out["roofline"]["measured_copy_GBs"] = copy_gbs
    out["roofline"]["frac_of_measured_copy"] = achieved / copy_gbs

    # ---- other precisions on the same system ----
    if not args.no_mixed:
        xa -= xa.mean()
        for label, prec in [("mixed_fp32", aar.AAR_MIXED_FP32), ("fp64_fp32hist", aar.AAR_FP64_FP32HIST)]:
            pm = inputs.Params(**{**prm.__dict__})
            pm.precision = prec
            sm = aar.Solver([prob], pm)
            dtm, rm, xm = timed_solves(sm, bt, args.steps, args.warmup)
            sm.close()
            xb = xm.cpu().numpy()
            err = oracle_sample_error(xb, args.n)
            xb -= xb.mean()
            out[label] = {"value": args.steps / dtm, "unit": "solves/s", "ms_per_step": dtm / args.steps * 1e3,
                          "iterations": rm["iterations"], "outer_steps": rm["outer_steps"],
                          "rel_residual": rm["rel_residual"], "status": rm["status"],
                          "speedup_vs_fp64": dt64 / dtm, "error_vs_oracle": err,
                          "rel_diff_vs_fp64_gpu": float(np.linalg.norm(xa - xb) / np.linalg.norm(xa))}

    # ---- batched: 512 shifted periodic Helmholtz systems, one call ----
    if not args.no_batched:
        out["batched"] = run_batched(args)

    # ---- CPU oracle baseline (bounded sample) ----
    if not args.no_cpu_baseline:
        import oracle
        k = args.cpu_sample_iters
        t0 = time.perf_counter()
        oracle.aar_solve(prob, b, m=prm.m, p=prm.p, tol=1e-30, max_iter=k)
        dtc = time.perf_counter() - t0
        iters_full = None
        if os.path.exists(GOLDEN):
            g = json.load(open(GOLDEN))
            key = f"periodic_poisson_r6_{args.n}"
            if key in g:
                iters_full = g[key]["iterations"]
        basis = "oracle iterations to 1e-10 (tests/golden)" if iters_full else "GPU iteration count"
        iters_full = iters_full or r64["iterations"]
        out["cpu_baseline"] = {"value": 1.0 / (dtc / k * iters_full), "unit": "solves/s",
                               "cores": oracle.threads(), "kind": "oracle",
                               "sample": f"{k} AAR iterations of the same {args.n}^3 system ({dtc:.1f} s), "
                                         f"scaled by {iters_full} iterations per solve ({basis})"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
