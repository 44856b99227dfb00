"""Tune the stencil tile shapes of the evaluation grids on the current GPU.

Creates a solver for each grid shape of the evaluation workloads (which runs
the library's autotuner) with AAR_TUNE_CACHE pointing at an empty file and
AAR_TUNE_CACHE_WRITE at the output, so every shape is timed afresh and its
choice appended.  The library reads tuned_tiles.txt next to itself at
creation, so committing the output makes tile choices reproducible.

The batched engine uses one tile shape for all systems of a batch; with
--batched the shape is chosen by timing whole batched solves of the 512-system
Helmholtz workload for rows per thread {1, 2, 4} x z depth {4, 8, 16, 32}, and
the winner is appended as a batch line (grid fields 0 0 0).

Usage: python -m paper_1606_08740_amd.tune_tiles [--batched] [output path]
"""
import os
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def shapes():
    from paper_1606_08740_amd import inputs
    out = []
    for n in (32,):
        out.append(inputs.dirichlet_poisson_problem(n))
    for n in (192, 256):
        out.append(inputs.periodic_problem(n, 6))
    cd = inputs.dirichlet_poisson_problem(128)
    cd.velocity = inputs.convection_field(128, 4)
    out.append(cd)
    return out


def main(path):
    empty = tempfile.NamedTemporaryFile(delete=False)
    empty.close()
    os.environ["AAR_TUNE_CACHE"] = empty.name
    os.environ["AAR_TUNE_CACHE_WRITE"] = path
    if os.path.exists(path):
        os.remove(path)
    with open(path, "w") as f:
        f.write("# prec radius conv n0 n1 n2 rows_per_thread z_depth order pair  (prec 0 = FP64, 1 = FP32)\n")
    from paper_1606_08740_amd import aar, inputs
    for prob in shapes():
        for precision in (aar.AAR_FP64, aar.AAR_MIXED_FP32):
            s = aar.Solver([prob], inputs.Params(precision=precision))
            s.close()
            print(f"tuned n={prob.n} r={prob.radius} conv={prob.velocity is not None} precision={precision}",
                  flush=True)
    os.remove(empty.name)
    print(open(path).read())


def tune_batched(path):
    import time

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
        lines.append(f"{prec} {radius} 0 0 0 0 {best[1]} {best[2]} 0 0\n")
    with open(path, "a") as f:
        f.writelines(lines)
    print("".join(lines))


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "--batched"]
    out = args[0] if args else os.path.join(HERE, "tuned_tiles.txt")
    if "--batched" in sys.argv[1:]:
        tune_batched(out)
    else:
        main(out)
