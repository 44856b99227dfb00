"""Temporal blocks of the Richardson steps (one pass computes several
consecutive steps of the residual recursion, and the Anderson-step residual
with them) against one pass per step, and against the oracle.

The tile file fixes the one-point tile shape and the block depth (its last
field); the same grid is solved with depth 0 (one pass per step) and with
blocks of 2 .. 5 steps.  Per point the block computes each step with the
single pass's arithmetic, so iterates at caps inside and after cycles agree to
rounding (1e-14 of max |x| in FP64, 1e-6 in the mixed mode's FP32 inner
solves, where the compiler may contract a multiply-add differently in the two
kernels); FP64 full solves take the same number of iterations within a cycle.
Grids: Dirichlet 7-point with ragged tiles, a periodic radius-2 grid narrower
than the block's halo, upwind convection, the FP32 inner solves of the mixed
mode, and p = 2, 3 where the last block holds only the Anderson residual.
"""
import numpy as np
import pytest

import oracle
from paper_1606_08740_amd import aar, inputs
from tests.gpu_util import gpu_solve, params, say
from tests.test_gpu_fp64 import cd_problem

pytestmark = pytest.mark.gpu

CASES = [
    # name, problem, (rows per thread, z depth), depths, params
    ("dirichlet_r1", inputs.Problem(n=(40, 33, 29), h=(1 / 41, 1 / 34, 1 / 30), bc=(0, 0, 0), radius=1),
     (2, 8), (2, 3, 5), dict(m=7, p=6)),
    ("periodic_r2_narrow", inputs.Problem(n=(50, 20, 17), h=(0.02, 0.05, 1 / 17), bc=(1, 1, 1), radius=2, shift=0.6),
     (4, 6), (2, 4), dict(m=7, p=6)),
    ("upwind_m10_p4", cd_problem((66, 35, 21)), (2, 8), (3,), dict(m=10, p=4)),
    ("mixed_bc_p3", inputs.Problem(n=(30, 18, 25), h=(0.03, 0.05, 0.04), bc=(1, 0, 0), radius=1, shift=0.1),
     (1, 4), (2,), dict(m=4, p=3)),
    ("p2_fk_only", inputs.Problem(n=(24, 24, 24), h=(1 / 25,) * 3, bc=(0, 0, 0), radius=2), (2, 8), (4,),
     dict(m=3, p=2)),
]


def _tiles(tmp_path, prob, ry, cz, depth):
    conv = 1 if prob.velocity is not None else 0
    f = tmp_path / f"tiles_{depth}.txt"
    n = prob.n
    f.write_text(f"0 {prob.radius} {conv} {n[0]} {n[1]} {n[2]} {ry} {cz} 0 0 {depth}\n"
                 f"1 {prob.radius} {conv} {n[0]} {n[1]} {n[2]} {ry} {cz} 0 0 {depth}\n")
    return str(f)


@pytest.mark.parametrize("name,prob,shape,depths,kw", CASES, ids=[c[0] for c in CASES])
def test_blocks_match_single_steps_and_oracle(name, prob, shape, depths, kw, tmp_path, monkeypatch):
    b = inputs.normal(23, 0, prob.size)
    p = kw["p"]
    for prec in (aar.AAR_FP64, aar.AAR_MIXED_FP32):
        ref_x, ref_it = {}, None
        for depth in (0,) + tuple(depths):
            monkeypatch.setenv("AAR_TUNE_CACHE", _tiles(tmp_path, prob, *shape, depth))
            for K in (p - 1, p, p + 1, 2 * p + 3):
                say(f"tblock {name} precision={prec} depth={depth} K={K}")
                x, res, _ = gpu_solve(prob, params(max_iter=K, tol=1e-30, precision=prec, **kw), b)
                assert res["status"] == aar.AAR_NOT_CONVERGED and res["iterations"] == K, res
                if depth == 0:
                    ref_x[K] = x
                    if prec == aar.AAR_FP64:
                        o = oracle.aar_solve(prob, b, m=kw["m"], p=p, tol=1e-30, max_iter=K)["x"]
                        np.testing.assert_allclose(x, o, rtol=0, atol=1e-10 * np.abs(o).max())
                else:
                    # rounding of the iterate's type: the two kernels may contract
                    # a multiply-add differently (FP32: a few units in the last place)
                    rel = 1e-14 if prec == aar.AAR_FP64 else 1e-6
                    np.testing.assert_allclose(x, ref_x[K], rtol=0, atol=rel * np.abs(ref_x[K]).max(),
                                               err_msg=f"depth {depth} K={K}")
            say(f"tblock {name} precision={prec} depth={depth} full solve")
            x, res, _ = gpu_solve(prob, params(tol=1e-10, precision=prec, **kw), b)
            assert res["status"] == aar.AAR_OK, res
            assert oracle.relative_residual(prob, b, x) < 1e-10
            if ref_it is None:
                ref_it = res["iterations"]
            elif prec == aar.AAR_FP64:
                assert abs(res["iterations"] - ref_it) <= p
