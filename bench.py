"""Benchmark of the MI355X AAR solver: solves/s at 1e-10 relative residual.

A step is one complete AAR solve (every stage of the iteration: fused
Richardson sweeps, Anderson residual and Gram reduction, pseudoinverse
solve, update; plus FP64 refinement in mixed mode) of one seeded synthetic
system whose right-hand side and solver workspace are already resident in
HBM.  The headline (`value`) is the largest single-grid workload at the
paper's arithmetic: periodic Poisson 256^3, 12th-order central differences
(37-point stencil), 64 Gaussian charges minus their mean, Jacobi
preconditioner, omega = beta = 0.6, m = 7, p = 6, tol 1e-10, FP64.

Beside it, in the same JSON line, every other evaluation workload and mode,
each with solves/s, iterations, the speedup over FP64 on the same system and
the error against the oracle's stored FP64 solution:
  c3_256   the headline grid in mixed precision (FP32 inner AAR + FP64
           refinement; FP32 or bfloat16 history) and FP64 with an FP32 ring;
  c2_192   the same problem at 192^3 (FP64, mixed, FP64 + FP32 ring);
  c4_128   nonsymmetric convection-diffusion 128^3, m = 10, p = 4;
  c1_32    Dirichlet Poisson 32^3 at 1e-8 (FP64) and 1e-10 (FP64, mixed),
           reported as microseconds per iteration (launch-bound size);
  batched  512 periodic shifted Helmholtz systems of uneven sizes in one call:
           the paper's method in FP64 and, with the exact constant-mode
           deflation (not in the paper), FP64, mixed and FP64 + FP32 ring;
           each with a whole-call bandwidth figure;
  complex_helmholtz  the complex periodic Helmholtz problem of orbital-free
           DFT (the paper's P and Q), 72^3 and 144^3, complex FP64.
`roofline` covers the dominant kernel of the headline, the Richardson sweep:
algorithmic bytes per launch over the mean launch time measured with HIP
events on the solver's stream, against the 8 TB/s HBM peak.  Each solve also
gets an effective bandwidth: the method's algorithmic bytes per cycle (model
in cycle_bytes) times its cycles, over the solve time.  `cpu_baseline` times
the oracle (built -O3 -march=native on this host) on a bounded number of
iterations of the headline system and scales to solves/s with the oracle's
own iteration count.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "AAR solves/s and sweep HBM GB/s at 1e-10 rel-residual: mixed/batched vs FP64"
HBM_PEAK_GBS = 8000.0
# Oracle (FP64, CPU) solutions at full size, written by tests/golden/make_golden.py (oracle only).
GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_full_size.json")
# HBM traffic of the headline sweep kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs, scaled by a plain copy's counters; valid while the stencil sources and
# the grid's tile shape are those it was measured with.
PROFILE_DIR = os.path.join(ROOT, "profiles")
STENCIL_SRCS = [os.path.join(ROOT, "paper_1606_08740_amd", "csrc", f)
                for f in ("stencil_kernels.h", "stencil.hip", "stencil_narrow.hip", "stencil_f32.hip")]

FP64, MIXED, MIXED_BF16, FP64_FP32HIST, FP64_BF16HIST = 0, 1, 2, 3, 4
MODE_NAMES = {FP64: "fp64", MIXED: "mixed_fp32", MIXED_BF16: "mixed_fp32_bf16hist",
              FP64_FP32HIST: "fp64_fp32hist", FP64_BF16HIST: "fp64_bf16hist"}


def log(msg):
    """Progress on stderr (the JSON line is the only stdout output)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


def sweep_profile(n):
    """The machine-readable record of profiles/k_stencil*_sweep_fp64_r6_<n>.md, or None."""
    import glob
    import re
    for path in sorted(glob.glob(os.path.join(PROFILE_DIR, f"k_stencil*_sweep_fp64_r6_{n}.md"))):
        m = re.search(r"```json\n(.*?)\n```", open(path).read(), flags=re.S)
        if m:
            return json.loads(m.group(1))
    return None


def sweep_traffic(n):
    """Counter-measured bytes per sweep launch at n^3, or None when absent or
    stale (other stencil sources or another tile shape)."""
    rec = sweep_profile(n)
    if rec is None or rec.get("stencil_source_sha256_16") != stencil_sha() or rec.get("tile") != fp64_tile(n):
        return None
    return rec.get("traffic_bytes_per_launch")


def sweep_bytes_per_point(m, p):
    """Algorithmic bytes per point of one FP64 Richardson sweep launch,
    averaged over a cycle's p - 1 sweeps.  With the residual recursion
    (m + 1 >= p >= 2) the first sweep reads x and b and writes f (24 B), the
    others read f_j and write f_{j+1} (16 B); otherwise each reads x and b and
    writes x and f (32 B)."""
    if m + 1 >= p >= 2:
        return (3 * 8 + (p - 2) * 2 * 8) / (p - 1)
    return 32.0


def cycle_bytes(precision, m, p, fused_gram=False):
    """Algorithmic bytes per grid point of one AAR cycle (p iterations) of the
    given mode: every vector a pass must read or write, counted once.
      FP64: first sweep 2s + s_h, the others 2 s_h (recursion) or 3s + s_h;
        Anderson residual 2 s_h (recursion) or 2s + s_h; Gram (m + 1) s_h
        (fused into the residual pass: the slots it did not read); update x,
        m + 1 slots, q increments, x and one increment written.
      FP64 + FP32 ring: as FP64 with 4-byte slots and increments, the later
        sweeps and the residual over the ring only.
      Mixed: the inner FP32 cycles (FP32 iterate and ring, recursion); the
        FP64 refinement passes (a few per solve) are left out.
    Returns None for the bfloat16-history modes (not modelled)."""
    q = m // p
    rec = m + 1 >= p >= 2
    if precision == FP64:
        s = sh = sdx = 8
    elif precision == FP64_FP32HIST:
        s, sh, sdx = 8, 4, 4
    elif precision == MIXED:
        s = sh = sdx = 4
    else:
        return None
    if rec:
        sweeps = (2 * s + sh) + (p - 2) * 2 * sh
        resid = 2 * sh
        gram = (m - 1) * sh if fused_gram else (m + 1) * sh
    else:
        sweeps = (p - 1) * (3 * s + sh)
        resid = 2 * s + sh
        gram = m * sh if fused_gram else (m + 1) * sh
    update = s + (m + 1) * sh + q * sdx + s + sdx
    return sweeps + resid + gram + update


def complex_cycle_bytes(m, p):
    """Algorithmic bytes per point of one cycle of the complex iteration
    (16-byte values; every Richardson sweep reads x and b and writes x and f,
    the Anderson-step residual reads x and b and writes f, the Gram pass reads
    the m + 1 slots, the update reads x, the slots and the q increments and
    writes x and one increment)."""
    z, q = 16, m // p
    return (p - 1) * 4 * z + 3 * z + (m + 1) * z + (z + (m + 1) * z + q * z + 2 * z)


def run_complex(args):
    """The complex periodic Helmholtz problem of orbital-free DFT (the
    paper's P, Q and alpha; sixth-order FD) on one and on eight aluminium
    cells at h = 0.108 Bohr, complex FP64."""
    import numpy as np
    import torch
    from paper_1606_08740_amd import aar, inputs
    out = {}
    for n, cells in ((72, 1), (144, 2)):
        log(f"complex helmholtz n={n}")
        prob, s_im, b, prm = inputs.ofdft_helmholtz(n, cells=cells)
        bt = torch.as_tensor(b, device="cuda:0")
        s = aar.ComplexSolver(prob, prm, s_im)
        res = None
        for _ in range(max(args.warmup, 1)):
            res = s.solve(bt, torch.zeros_like(bt))
        xs = [torch.zeros_like(bt) for _ in range(args.side_steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for x in xs:
            res = s.solve(bt, x)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / args.side_steps
        s.close()
        x = xs[-1].cpu().numpy()
        cb = complex_cycle_bytes(prm.m, prm.p)
        gbs = prob.size * cb * (res["iterations"] / prm.p) / per / 1e9
        out[f"n{n}"] = {"workload": f"OF-DFT periodic Helmholtz (Eq. 7), {cells}^3 Al FCC cells, {n}^3 grid, "
                                    "h = 0.108 Bohr, sixth-order FD, Jacobi, m=7, p=6, tol 1e-10, complex FP64",
                        "value": 1.0 / per, "unit": "solves/s", "ms_per_solve": per * 1e3,
                        "iterations": res["iterations"], "status": res["status"],
                        "rel_residual": res["rel_residual"],
                        "error_vs_oracle": complex_sample_error(x, f"ofdft_helmholtz_{n}"),
                        "oracle_iterations": (golden(f"ofdft_helmholtz_{n}") or {}).get("iterations"),
                        "effective_GBs": gbs, "effective_frac_of_peak": gbs / HBM_PEAK_GBS,
                        "bytes_per_point_per_cycle": cb}
        del bt, xs
    return out


def csr_sweep_bytes(n, nnz, nnz_factors=0):
    """Algorithmic bytes of one sparse Richardson sweep: A's values, columns
    and row pointers once (12 nnz + 8 (n + 1)), x, b, the new x and f (32 n);
    block ILU(0) adds its factors once, values and columns (12 per entry
    inside the blocks)."""
    return 12 * nnz + 8 * (n + 1) + 32 * n + 12 * nnz_factors


def run_sparse(args):
    """General sparse A (the paper's Sec. 3.1 study of nonsymmetric systems,
    Jacobi and ILU(0); the block-Jacobi ILU(0) of Secs. 3.2-3.3): a 128^3
    seven-point reservoir matrix (heterogeneous permeability, upwind
    convection) standing in for the Matrix Market systems, the paper's
    parameters (omega = beta = 0.6, m = 9, p = 8), tol 1e-6, x0 = 1."""
    import numpy as np
    import torch
    from paper_1606_08740_amd import aar, inputs
    n3 = args.sparse_n
    log(f"sparse reservoir n={n3}^3")
    A = inputs.reservoir_matrix(n3, seed=40)
    prm = inputs.Params(omega=0.6, beta=0.6, m=9, p=8, tol=1e-6, max_iter=100000)
    b = inputs.normal(31, 1, A.n)
    bt = torch.as_tensor(b, device="cuda:0")
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    out = {"workload": f"reservoir matrix {n3}^3 (7-point two-point flux, log-normal permeability sigma 1.5, "
                       "upwind convection, no-flow boundaries), b ~ N(0,1), x0 = 1, omega=beta=0.6, m=9, p=8, "
                       "tol 1e-6, FP64",
           "rows": A.n, "nnz": A.nnz}
    for name, pc, nb in (("jacobi", aar.AAR_PRECOND_JACOBI, 1),
                         (f"block_ilu0_{args.sparse_blocks}", aar.AAR_PRECOND_ILU0, args.sparse_blocks)):
        t0 = time.perf_counter()
        s = aar.CsrSolver(A, prm, pc, nb)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        res = s.solve(bt, torch.ones_like(bt))
        xs = [torch.ones_like(bt) for _ in range(args.side_steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for x in xs:
            res = s.solve(bt, x)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / args.side_steps
        s.set_timing(True)
        s.solve(bt, torch.ones_like(bt))
        torch.cuda.synchronize()
        ms, launches = s.sweep_time()
        s.close()
        x = xs[-1].cpu().numpy()
        if pc == aar.AAR_PRECOND_ILU0:
            first = np.arange(nb + 1) * A.n // nb
            blk = np.searchsorted(first, rows, side="right") - 1
            nnz_f = int(((A.col >= first[blk]) & (A.col < first[blk + 1])).sum())
        else:
            nnz_f = 0
        sb = csr_sweep_bytes(A.n, A.nnz, nnz_f)
        sweep_us = 1e3 * ms / max(launches, 1)
        out[name] = {"value": 1.0 / per, "unit": "solves/s", "ms_per_solve": per * 1e3,
                     "setup_ms": t_setup * 1e3, "iterations": res["iterations"], "status": res["status"],
                     "rel_residual": res["rel_residual"],
                     "error_vs_oracle": sparse_sample_error(x, f"reservoir_128_{name}" if n3 == 128 else None),
                     "oracle_iterations": (golden(f"reservoir_128_{name}") or {}).get("iterations") if n3 == 128
                     else None,
                     "sweep_us": sweep_us, "sweep_bytes": sb,
                     "sweep_GBs": sb / (sweep_us * 1e-6) / 1e9,
                     "sweep_frac_of_peak": sb / (sweep_us * 1e-6) / 1e9 / HBM_PEAK_GBS}
        del xs
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="headline grid edge (periodic Poisson, radius 6)")
    ap.add_argument("--side-steps", type=int, default=3, help="timed solves per side measurement")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=120)
    ap.add_argument("--kernel-timing-solves", type=int, default=1)
    ap.add_argument("--sparse-n", type=int, default=128, help="grid edge of the sparse reservoir matrix")
    ap.add_argument("--sparse-blocks", type=int, default=1024, help="blocks of the block-Jacobi ILU(0)")
    ap.add_argument("--only", choices=["headline", "c1", "c2", "c3", "c4", "c5", "complex", "sparse"],
                    help="run one part only and print its JSON object (for profiling)")
    ap.add_argument("--precision", type=int, choices=[0, 1, 2, 3, 4],
                    help="with --only: the one precision mode to time")
    ap.add_argument("--batched-count", type=int, default=512)
    ap.add_argument("--batched-steps", type=int, default=2)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scale for the FETCH_SIZE / WRITE_SIZE counters)")
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


def golden(key):
    if not os.path.exists(GOLDEN):
        return None
    return json.load(open(GOLDEN)).get(key)


def complex_sample_error(x, key):
    """Max |x - x_oracle| over the 64 stored sample points of the complex
    oracle's solution (tests/golden), divided by that solution's RMS; None
    without a stored entry."""
    g = golden(key)
    if g is None:
        return None
    ref = [complex(r, i) for r, i in zip(g["sample_re"], g["sample_im"])]
    return max(abs(x[i] - v) for i, v in zip(g["sample_index"], ref)) / g["x_rms"]


def sparse_sample_error(x, key):
    """The same for the sparse system's stored oracle solution."""
    g = golden(key) if key else None
    if g is None:
        return None
    return max(abs(x[i] - v) for i, v in zip(g["sample_index"], g["sample_x"])) / g["x_rms"]


def oracle_sample_error(x, n, key=None):
    """Max |x - x_oracle| over the 64 seeded sample points stored in the golden
    file (the oracle's FP64 solution of the same system, mean-free when the
    system is singular periodic), divided by the RMS of the oracle's solution;
    None when no stored solution exists for this system."""
    import numpy as np
    g = golden(key or f"periodic_poisson_r6_{n}")
    if g is None or int(np.prod(g["n"])) != x.size:
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


def fused_gram_used(n, m, radius=6):
    """Whether the FP64 Anderson-residual pass forms the Gram products itself
    (paired tile, 8 or fewer waves, m = 7) for this grid."""
    tile = fp64_tile(n, radius)
    return tile is not None and 0 < tile["pair"] <= 2 and m == 7


def run_modes(w, key, modes, steps, warmup, n=None):
    """Solve the workload's system in each mode (a precision, or a pair
    (precision, flags) recorded as "<mode>_recycle" for the carried history);
    returns {mode: record}, with the speedup over FP64 when FP64 is among the
    modes."""
    import torch
    from paper_1606_08740_amd import aar, inputs
    prob, b = w.problems[0], w.b[0]
    bt = torch.as_tensor(b, device="cuda:0")
    out, t64 = {}, None
    for mode in modes:
        prec, flags = mode if isinstance(mode, tuple) else (mode, 0)
        name = MODE_NAMES[prec] + ("_recycle" if flags & aar.AAR_FLAG_RECYCLE_HISTORY else "")
        log(f"{w.name} {name}")
        pm = inputs.Params(**{**w.params.__dict__})
        pm.precision = prec
        pm.flags |= flags
        s = aar.Solver([prob], pm)
        dt, r, xt = timed_solves(s, bt, steps, warmup)
        s.close()
        x = xt.cpu().numpy()
        per = dt / steps
        rec = {"value": 1.0 / per, "unit": "solves/s", "ms_per_solve": per * 1e3, "iterations": r["iterations"],
               "outer_steps": r["outer_steps"], "rel_residual": r["rel_residual"], "status": r["status"],
               "error_vs_oracle": oracle_sample_error(x, n or 0, key)}
        cb = cycle_bytes(prec, pm.m, pm.p, fused_gram=(prec == FP64 and n is not None and fused_gram_used(n, pm.m)))
        if cb is not None and r["iterations"] > 0:
            gbs = prob.size * cb * (r["iterations"] / pm.p) / per / 1e9
            rec["effective_GBs"] = gbs
            rec["effective_frac_of_peak"] = gbs / HBM_PEAK_GBS
            rec["bytes_per_point_per_cycle"] = cb
        if prec == FP64 and not flags:
            t64 = per
        out[name] = rec
        del xt
    if t64 is not None:
        for name, rec in out.items():
            rec["speedup_vs_fp64"] = t64 / (rec["ms_per_solve"] * 1e-3)
    del bt
    return out


def run_batched(args, modes=None):
    """The batched workload: 512 shifted periodic Helmholtz systems of uneven
    sizes solved by one aar_solve_batched call, in the paper's plain method
    (FP64) and with the exact constant-mode deflation (FP64, mixed, FP64 +
    FP32 ring).  Whole-call bandwidth: sum over systems of points x cycles x
    the mode's bytes per point and cycle, over the call time."""
    import numpy as np
    import torch
    from paper_1606_08740_amd import aar, inputs
    wb = inputs.workload(5, count=args.batched_count)
    bb = torch.as_tensor(np.concatenate(wb.b), device="cuda:0")
    sizes = np.array([p.size for p in wb.problems], dtype=np.float64)
    res_out = {"workload": f"{args.batched_count} periodic shifted Helmholtz systems, 8th-order "
                           "central FD (25-point), n ~ U{16..96}, sigma ~ U(0,10), b ~ N(0,1), tol 1e-10",
               "points": int(sizes.sum()), "min_shift": float(min(p.shift for p in wb.problems))}
    runs = modes or [("fp64_plain", FP64, 0), ("fp64", FP64, aar.AAR_FLAG_DEFLATE_CONSTANT),
                     ("mixed_fp32", MIXED, aar.AAR_FLAG_DEFLATE_CONSTANT),
                     ("fp64_fp32hist", FP64_FP32HIST, aar.AAR_FLAG_DEFLATE_CONSTANT)]
    for label, prec, flags in runs:
        log(f"batched {label}")
        pb = inputs.Params(**{**wb.params.__dict__})
        pb.precision = prec
        pb.flags = flags
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
        its = np.array([r["iterations"] for r in res], dtype=np.float64)
        rec = {"value": args.batched_count / dtb, "unit": "solves/s", "ms_per_call": dtb * 1e3,
               "deflated": bool(flags & aar.AAR_FLAG_DEFLATE_CONSTANT),
               "converged": int(sum(r["status"] == 0 for r in res)),
               "iterations_total": int(its.sum()), "iterations_max": int(its.max()),
               "max_rel_residual": float(max(r["rel_residual"] for r in res))}
        cb = cycle_bytes(prec, pb.m, pb.p)
        if cb is not None:
            gbs = float((sizes * (its / pb.p)).sum()) * cb / dtb / 1e9
            rec["effective_GBs"] = gbs
            rec["effective_frac_of_peak"] = gbs / HBM_PEAK_GBS
            rec["bytes_per_point_per_cycle"] = cb
        res_out[label] = rec
    if "fp64" in res_out:
        for label, _, _ in runs:
            res_out[label]["speedup_vs_fp64_deflated"] = res_out[label]["value"] / res_out["fp64"]["value"]
    del bb
    return res_out


def headline(args):
    """The headline FP64 solve, its sweep-kernel roofline and error."""
    import numpy as np
    import torch
    from paper_1606_08740_amd import aar, inputs
    w = inputs.workload(3, n=args.n, precision=FP64) if args.n != 192 else inputs.workload(2)
    prob, b = w.problems[0], w.b[0]
    N = prob.size
    prm = w.params
    prm.precision = FP64
    bt = torch.as_tensor(b, device="cuda:0")
    log(f"headline {w.name} fp64")
    s64 = aar.Solver([prob], prm)
    dt64, r64, x64 = timed_solves(s64, bt, args.steps, args.warmup)
    # kernel timing: one HIP event pair around each cycle's p - 1 consecutive
    # sweep launches, on the solver's stream (one extra solve)
    s64.set_timing(True)
    for _ in range(args.kernel_timing_solves):
        xt = torch.zeros_like(bt)
        s64.solve(bt, xt)
    ms_tot, launches = s64.sweep_time()
    s64.set_timing(False)
    s64.close()
    sweep_us = ms_tot / max(launches, 1) * 1e3
    bpp = sweep_bytes_per_point(prm.m, prm.p)
    sweep_bytes = bpp * N
    achieved = sweep_bytes / (sweep_us * 1e-6) / 1e9
    tile = fp64_tile(args.n)
    per = dt64 / args.steps
    cb = cycle_bytes(FP64, prm.m, prm.p, fused_gram=fused_gram_used(args.n, prm.m))
    eff = N * cb * (r64["iterations"] / prm.p) / per / 1e9
    key = f"periodic_poisson_r6_{args.n}"
    x = x64.cpu().numpy()
    out = {
        "dt": dt64, "r": r64, "N": N,
        "config": {"workload": f"periodic Poisson {args.n}^3, 12th-order central FD (37-point), "
                               "64 Gaussian charges minus mean, Jacobi, omega=beta=0.6, m=7, p=6, "
                               "tol 1e-10, FP64",
                   "grid": [args.n] * 3, "radius": 6, "m": prm.m, "p": prm.p, "tol": prm.tol, "precision": "fp64",
                   "tile": tile},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": sweep_traffic(args.n),
                     "kernel": "Richardson sweep (FP64, radius 6): a cycle's first from x and b, the others "
                               "by the residual recursion f_{j+1} = f_j - omega D^-1 A f_j",
                     "bytes_per_point": bpp, "bytes_per_launch": sweep_bytes, "mean_launch_us": sweep_us,
                     "launches": launches},
        "solve": {"effective_GBs": eff, "effective_frac_of_peak": eff / HBM_PEAK_GBS,
                  "bytes_per_point_per_cycle": cb,
                  "error_vs_oracle": oracle_sample_error(x, args.n, key),
                  "oracle_iterations": (golden(key) or {}).get("iterations")},
    }
    del bt, x64
    return out, w


def cpu_baseline(args, w):
    """The oracle, built -O3 -march=native here, on a bounded sample of the
    headline system (the first cpu_sample_iters iterations), scaled to
    solves/s by the oracle's own iteration count."""
    import oracle
    prob, b, prm = w.problems[0], w.b[0], w.params
    log("cpu baseline")
    with tempfile.TemporaryDirectory() as d:
        flags = oracle.load_native(d)
        k = args.cpu_sample_iters
        t0 = time.perf_counter()
        oracle.aar_solve(prob, b, m=prm.m, p=prm.p, tol=1e-30, max_iter=k)
        dtc = time.perf_counter() - t0
        cores = oracle.threads()
    g = golden(f"periodic_poisson_r6_{args.n}")
    iters_full = g["iterations"] if g else None
    basis = "the oracle's iterations to 1e-10 (tests/golden)" if iters_full else "no stored count: per iteration"
    return {"value": 1.0 / (dtc / k * iters_full) if iters_full else k / dtc,
            "unit": "solves/s" if iters_full else "iterations/s", "cores": cores, "kind": "oracle",
            "build": "gcc " + " ".join(flags),
            "sample": f"{k} AAR iterations of the {args.n}^3 headline system ({dtc:.1f} s on {cores} threads), "
                      f"scaled by {iters_full} iterations per solve ({basis})"}


def c1(args):
    """32^3 Dirichlet Poisson: launch-bound; microseconds per iteration."""
    from paper_1606_08740_amd import inputs
    steps = max(args.side_steps * 10, 20)
    out = {}
    for label, tol, modes in [("tol_1e-8", 1e-8, [FP64]), ("tol_1e-10", 1e-10, [FP64, MIXED, FP64_FP32HIST])]:
        w = inputs.workload(1, tol=tol)
        key = f"dirichlet_poisson_7pt_32_tol{'1e-8' if tol == 1e-8 else '1e-10'}"
        r = run_modes(w, key, modes, steps, 3)
        for rec in r.values():
            rec["us_per_iteration"] = rec["ms_per_solve"] * 1e3 / max(rec["iterations"], 1)
            rec.pop("effective_GBs", None)
            rec.pop("effective_frac_of_peak", None)
        r["oracle_iterations"] = (golden(key) or {}).get("iterations")
        out[label] = r
    out["note"] = "working set in L2 / Infinity Cache: launch latency, not HBM, bounds it; reported per iteration"
    # beta / p chosen by timed trial solves, then the full solve with them
    import torch
    from paper_1606_08740_amd import aar
    w = inputs.workload(1, tol=1e-10)
    prob, b = w.problems[0], w.b[0]
    bt = torch.as_tensor(b, device="cuda:0")
    betas, ps = [0.3, 0.6, 1.0, 1.3], [2, 4, 6, 8]
    log("c1 parameter selection")
    t0 = time.perf_counter()
    beta, p, scores = aar.aar_select_parameters(aar.make_problem(prob), aar.make_params(w.params), bt.data_ptr(),
                                                 betas, ps, 96)
    t_sel = time.perf_counter() - t0
    pm = inputs.Params(**{**w.params.__dict__})
    pm.beta, pm.p = beta, p
    sv = aar.Solver([prob], pm)
    dt, r, _ = timed_solves(sv, bt, steps, 3)
    sv.close()
    out["parameter_selection"] = {
        "candidates": {"beta": betas, "p": ps}, "trial_iterations": 96, "selection_seconds": t_sel,
        "chosen": {"beta": beta, "p": p}, "ms_per_solve": dt / steps * 1e3, "iterations": r["iterations"],
        "status": r["status"], "speedup_vs_default": out["tol_1e-10"]["fp64"]["ms_per_solve"] / (dt / steps * 1e3)}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch
    from paper_1606_08740_amd import inputs

    assert torch.cuda.is_available(), "bench needs a GPU"
    steps, warm = args.side_steps, 1
    if args.only in ("c2", "c3", "c4"):
        w = {"c2": lambda: inputs.workload(2), "c3": lambda: inputs.workload(3, precision=FP64),
             "c4": lambda: inputs.workload(4, precision=FP64)}[args.only]()
        key = {"c2": "periodic_poisson_r6_192", "c3": "periodic_poisson_r6_256",
               "c4": "convection_diffusion_upwind_128"}[args.only]
        modes = [args.precision] if args.precision is not None else [FP64, MIXED, FP64_FP32HIST]
        print(json.dumps(run_modes(w, key, modes, args.steps, args.warmup, n=w.problems[0].n[0])))
        return
    if args.only == "c1":
        print(json.dumps(c1(args)))
        return
    if args.only == "complex":
        print(json.dumps(run_complex(args)))
        return
    if args.only == "sparse":
        print(json.dumps(run_sparse(args)))
        return
    if args.only == "c5":
        modes = None
        if args.precision is not None:
            from paper_1606_08740_amd import aar
            modes = [(MODE_NAMES[args.precision], args.precision, aar.AAR_FLAG_DEFLATE_CONSTANT)]
        print(json.dumps(run_batched(args, modes)))
        return

    h, w = headline(args)
    r64 = h["r"]
    out = {
        "metric": METRIC,
        "value": args.steps / h["dt"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["dt"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": h["config"],
        "iterations": r64["iterations"],
        "rel_residual": r64["rel_residual"],
        "status": r64["status"],
        "roofline": h["roofline"],
        "solve": h["solve"],
    }
    if args.only == "headline":
        print(json.dumps(out))
        return
    out["roofline"]["measured_copy_GBs"] = copy_gbs = measured_copy_gbs()
    out["roofline"]["frac_of_measured_copy"] = out["roofline"]["achieved"] / copy_gbs

    # ---- the headline grid in the other modes ----
    from paper_1606_08740_amd import aar
    rec_flag = aar.AAR_FLAG_RECYCLE_HISTORY
    c3 = run_modes(w, f"periodic_poisson_r6_{args.n}", [MIXED, (MIXED, rec_flag), MIXED_BF16, FP64_FP32HIST], steps,
                   warm, n=args.n)
    t64 = h["dt"] / args.steps
    for rec in c3.values():
        rec["speedup_vs_fp64"] = t64 / (rec["ms_per_solve"] * 1e-3)
    c3["fp64"] = {"value": 1.0 / t64, "unit": "solves/s", "ms_per_solve": t64 * 1e3,
                  "iterations": r64["iterations"], "error_vs_oracle": h["solve"]["error_vs_oracle"],
                  "effective_GBs": h["solve"]["effective_GBs"], "speedup_vs_fp64": 1.0}
    out[f"c3_{args.n}"] = c3
    del w
    # ---- the other evaluation workloads ----
    if args.n != 192:
        w2 = inputs.workload(2)
        out["c2_192"] = run_modes(w2, "periodic_poisson_r6_192", [FP64, MIXED, (MIXED, rec_flag), FP64_FP32HIST],
                                  steps, warm, n=192)
        del w2
    w4 = inputs.workload(4, precision=FP64)
    out["c4_128"] = run_modes(w4, "convection_diffusion_upwind_128", [FP64, MIXED, (MIXED, rec_flag), FP64_FP32HIST],
                              steps, warm, n=128)
    del w4
    out["c1_32"] = c1(args)
    out["batched"] = run_batched(args)
    out["complex_helmholtz"] = run_complex(args)
    out["sparse"] = run_sparse(args)

    # ---- CPU oracle baseline (bounded sample) ----
    if not args.no_cpu_baseline:
        wc = inputs.workload(3, n=args.n, precision=FP64) if args.n != 192 else inputs.workload(2)
        out["cpu_baseline"] = cpu_baseline(args, wc)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
