"""Tune the stencil tile shapes and temporal-block depths of the evaluation
grids on the current GPU, by timing whole solves.

The library's own autotuner (run by aar_create for a grid the tile file does
not list) times the Richardson sweep of each candidate shape and then, for a
one-point shape of radius <= 2, the block depth of the cycle's later steps.
A sweep-only objective can pick a shape that is slower over a whole cycle
(the Anderson-residual pass, which forms the Gram products itself in the
paired layout, and the update depend on it too), so this script times whole
solves instead: for each evaluation grid and precision it writes each
candidate as the grid's only tile line, solves the workload's system once to
warm up and then `--reps` times, and keeps the fastest.  The winners replace
their grids' lines in the output tile file (one line per grid and precision:
"prec radius conv n0 n1 n2 rows_per_thread z_depth order pair depth"); the
file's other lines are kept.  The library reads the file next to itself, so
committed choices are reproducible.

The batched engine uses one tile shape for all systems of a batch; with
--batched the shape is chosen by timing whole batched solves of the
512-system Helmholtz workload for rows per thread {1, 2, 4} x z depth
{4, 8, 16, 32}, and the winner replaces the batch line (grid fields
0 0 0).

Usage: python -m paper_1606_08740_amd.tune_tiles [--batched] [--reps K] [--grids c1,c2,c3,c4] [output path]
"""
import os
import sys
import tempfile
import time

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = ("# prec radius conv n0 n1 n2 rows_per_thread z_depth order pair depth  (prec 0 = FP64, 1 = FP32, "
          "2 = complex FP64 sweep, timed at creation; grid 0 0 0: the batched engine; depth: temporal block of "
          "recursion steps, 0 = one pass per step)\n")


def workloads():
    """(label, workload) of the evaluation grids: 32^3 Dirichlet, 192^3 and
    256^3 periodic radius 6, 128^3 convection-diffusion."""
    from paper_1606_08740_amd import inputs
    return [("c1", lambda: inputs.workload(1, tol=1e-10)), ("c2", lambda: inputs.workload(2)),
            ("c3", lambda: inputs.workload(3, precision=0)), ("c4", lambda: inputs.workload(4, precision=0))]


def candidates(prob, f64):
    """Tile shapes tried for one grid: one-point tiles (rows {1, 2, 4} x z
    depths, along x or (small grids) along z first, and with temporal blocks
    of 2, 3 or 5 steps where the radius allows),
    and paired tiles of 4 and 8 waves (16 too in FP32) with both z orders."""
    n = prob.n
    out = []
    small = n[2] <= 64
    depths = [2, 4, 8, 16, 32] if small else [16, 28, 32, 64]
    for ry in (1, 2, 4):
        for cz in depths:
            # small grids: also tiles numbered along z first (more z chunks
            # per XCD), which matter when the launches are latency-bound
            for order in ((0, 2) if small else (0,)):
                out.append((ry, cz, order, 0, 0))
            if prob.radius <= 2 and cz >= 4:
                for tb in (2, 3, 5):
                    out.append((ry, cz, 0, 0, tb))
    if n[0] % 2 == 0 and prob.velocity is None:
        pairs = [(1, 1), (2, 1), (1, 2)] + ([] if f64 else [(2, 2), (1, 3)])
        for ry, pair in pairs:
            for cz in depths:
                for order in (0, 1):
                    out.append((ry, cz, order, pair, 0))
    return out


def merge_lines(old_text, new_lines):
    """The tile file after tuning: the header, then the old file's lines
    whose grid and precision (the first six fields) were not tuned again, in
    their order, then the new lines.  Batch and complex lines, and grids left
    out of this run, are kept."""
    key = lambda line: tuple(line.split()[:6])
    fresh = {key(line) for line in new_lines}
    kept = [line if line.endswith("\n") else line + "\n" for line in old_text.splitlines()
            if line.strip() and not line.startswith("#") and key(line) not in fresh]
    return HEADER + "".join(kept) + "".join(new_lines)


def time_solve(prob, b, params, reps):
    import torch
    from paper_1606_08740_amd import aar
    s = aar.Solver([prob], params)
    bt = torch.as_tensor(b, device="cuda:0")
    s.solve(bt, torch.zeros_like(bt))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.solve(bt, torch.zeros_like(bt))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    s.close()
    return dt


def main(path, reps, grids):
    from paper_1606_08740_amd import aar, inputs
    lines = []
    for label, make in workloads():
        if grids and label not in grids:
            continue
        w = make()
        prob, b = w.problems[0], w.b[0]
        conv = 1 if prob.velocity is not None else 0
        key = f"{prob.radius} {conv} {prob.n[0]} {prob.n[1]} {prob.n[2]}"
        for prec, precision in ((0, aar.AAR_FP64), (1, aar.AAR_MIXED_FP32)):
            best = None
            for ry, cz, order, pair, tb in candidates(prob, prec == 0):
                line = f"{prec} {key} {ry} {cz} {order} {pair} {tb}\n"
                tile = tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False)
                tile.write(line)
                tile.close()
                os.environ["AAR_TUNE_CACHE"] = tile.name
                pm = inputs.Params(**{**w.params.__dict__})
                pm.precision = precision
                dt = time_solve(prob, b, pm, reps)
                os.remove(tile.name)
                print(f"{label} prec={prec} tile=({ry},{cz},{order},{pair},{tb}): {dt * 1e3:.3f} ms", flush=True)
                if best is None or dt < best[0]:
                    best = (dt, line)
            lines.append(best[1])
            print(f"{label} prec={prec} best: {best[1].strip()} ({best[0] * 1e3:.3f} ms)", flush=True)
    old = open(path).read() if os.path.exists(path) else ""
    with open(path, "w") as f:
        f.write(merge_lines(old, lines))
    print(open(path).read())


def tune_batched(path):
    import numpy as np
    import torch

    from paper_1606_08740_amd import aar, inputs
    wb = inputs.workload(5)
    bb = torch.as_tensor(np.concatenate(wb.b), device="cuda:0")
    radius = wb.problems[0].radius
    lines = []
    for precision in (aar.AAR_FP64, aar.AAR_MIXED_FP32):
        prec = 0 if precision == aar.AAR_FP64 else 1
        best = None
        for ry in (1, 2, 4):
            for cz in (4, 8, 16, 32):
                tile = tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False)
                tile.write(f"{prec} {radius} 0 0 0 0 {ry} {cz} 0 0\n")
                tile.close()
                os.environ["AAR_TUNE_CACHE"] = tile.name
                pb = inputs.Params(**{**wb.params.__dict__})
                pb.precision = precision
                s = aar.Solver(wb.problems, pb)
                s.solve_batched(bb, torch.zeros_like(bb))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.solve_batched(bb, torch.zeros_like(bb))
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                s.close()
                os.remove(tile.name)
                print(f"batched precision={precision} rows={ry} depth={cz}: {dt * 1e3:.1f} ms", flush=True)
                if best is None or dt < best[0]:
                    best = (dt, ry, cz)
        lines.append(f"{prec} {radius} 0 0 0 0 {best[1]} {best[2]} 0 0 0\n")
    old = open(path).read() if os.path.exists(path) else ""
    with open(path, "w") as f:
        f.write(merge_lines(old, lines))
    print("".join(lines))


if __name__ == "__main__":
    args = sys.argv[1:]
    reps, grids, rest = 2, None, []
    i = 0
    while i < len(args):
        if args[i] == "--reps":
            reps = int(args[i + 1])
            i += 2
        elif args[i] == "--grids":
            grids = set(args[i + 1].split(","))
            i += 2
        else:
            rest.append(args[i])
            i += 1
    out = [a for a in rest if a != "--batched"]
    path = out[0] if out else os.path.join(HERE, "tuned_tiles.txt")
    if "--batched" in rest:
        tune_batched(path)
    else:
        main(path, reps, grids)
