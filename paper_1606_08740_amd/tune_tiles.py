"""Tune the stencil tile shapes of the evaluation grids on the current GPU.

Creates a solver for each grid shape of the evaluation workloads (which runs
the library's autotuner) with AAR_TUNE_CACHE pointing at an empty file and
AAR_TUNE_CACHE_WRITE at the output, so every shape is timed afresh and its
choice appended.  The library reads tuned_tiles.txt next to itself at
creation, so committing the output makes tile choices reproducible.

Usage: python -m paper_1606_08740_amd.tune_tiles [output path]
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


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "tuned_tiles.txt"))
