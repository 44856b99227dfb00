"""GPU parity of the Moore-Penrose branch of the m x m solve (Sec. 3.2; the
footnote to Eq. 5) and of periodic axes shorter than the stencil.

The one-wave solve takes a Cholesky shortcut when a bound proves every
eigenvalue of F^T F above the pseudoinverse threshold, else a Jacobi
eigendecomposition that drops eigenvalues <= l lambda_max 2^-52.  These tests
  * force the eigendecomposition (AAR_FLAG_FORCE_PINV) on the same grids and
    iteration caps as the ordinary iterate parity, element by element against
    the oracle (which always takes the eigendecomposition);
  * drive the solve into a rank-deficient history: with b one sine
    eigenmode of the Dirichlet Laplacian, every f_j is a multiple of that mode
    (D is constant), so all columns of F_k are parallel and the kept rank is
    1; the iterates at caps p, p + 1 and 3p + 2 and the rank kept at the
    first Anderson step are compared with the oracle's, on the register
    (m <= 8) and LDS (m > 8) paths of the solve, and the kept rank is
    checked to be below l (the eigendecomposition truncated);
  * read the rank log to check which branch ran.
"""
import numpy as np
import pytest

import oracle
from paper_1606_08740_amd import aar, inputs
from tests.gpu_util import params, say, to_dev
from tests.test_gpu_fp64 import ITER_CASES

pytestmark = pytest.mark.gpu


def solve_logged(prob, prm, b):
    """Solve through the C ABI; returns x, result, residual log, rank log."""
    import torch
    s = aar.Solver([prob], prm)
    bt = to_dev(b)
    xt = torch.zeros_like(bt)
    res = s.solve(bt, xt)
    torch.cuda.synchronize()
    out = (xt.cpu().numpy(), res, s.residual_log(), s.rank_log())
    s.close()
    return out


@pytest.mark.parametrize("name,prob,kw", ITER_CASES, ids=[c[0] for c in ITER_CASES])
def test_forced_pinv_iterates_match_oracle(name, prob, kw):
    b = inputs.normal(5, 0, prob.size)
    p, m = kw["p"], kw["m"]
    for K in sorted({max(p - 1, 1), p, p + 1, 3 * p + 2}):
        say(f"forced pinv {name} K={K}")
        prm = params(max_iter=K, tol=1e-30, flags=aar.AAR_FLAG_FORCE_PINV | aar.AAR_FLAG_RECORD_RESIDUALS, **kw)
        x, res, log, ranks = solve_logged(prob, prm, b)
        ref = oracle.aar_solve(prob, b, m=m, p=p, tol=1e-30, max_iter=K, trace_cap=1000)
        assert res["status"] == aar.AAR_NOT_CONVERGED and res["iterations"] == K
        np.testing.assert_allclose(x, ref["x"], rtol=0, atol=1e-10 * np.abs(ref["x"]).max(), err_msg=f"K={K}")
        # one log entry per Anderson step reached; each kept rank is between
        # 0 and l = min(k, m) (the eigendecomposition ran: the Cholesky
        # shortcut always reports l)
        steps = K // p
        assert len(ranks) == len(log) == steps
        for t in range(steps):
            k = (t + 1) * p - 1
            assert 0 <= ranks[t] <= min(k, m)


def sine_mode(n, a, b_, c):
    """sin(a pi x) sin(b pi y) sin(c pi z) on the Dirichlet grid x = (i+1) h."""
    h = 1.0 / (n + 1)
    t = (np.arange(n) + 1) * h
    sx, sy, sz = np.sin(a * np.pi * t), np.sin(b_ * np.pi * t), np.sin(c * np.pi * t)
    return (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).ravel()


RANK1_CASES = [
    ("register_solve_m7", 20, (1, 2, 1), dict(m=7, p=6)),
    ("lds_solve_m9", 18, (2, 1, 3), dict(m=9, p=4)),
    ("p1_m5", 16, (1, 1, 2), dict(m=5, p=1)),
]


@pytest.mark.parametrize("force", [0, aar.AAR_FLAG_FORCE_PINV], ids=["auto", "forced"])
@pytest.mark.parametrize("name,n,mode,kw", RANK1_CASES, ids=[c[0] for c in RANK1_CASES])
def test_rank_deficient_eigenmode_matches_oracle(name, n, mode, kw, force):
    prob = inputs.dirichlet_poisson_problem(n)
    b = sine_mode(n, *mode)
    p, m = kw["p"], kw["m"]
    for K in sorted({p, p + 1, 3 * p + 2}):
        say(f"rank-1 eigenmode {name} K={K} force={force}")
        prm = params(max_iter=K, tol=1e-30, flags=aar.AAR_FLAG_RECORD_RESIDUALS | force, **kw)
        x, res, log, ranks = solve_logged(prob, prm, b)
        ref = oracle.aar_solve(prob, b, m=m, p=p, tol=1e-30, max_iter=K, trace_cap=1000)
        assert res["status"] == aar.AAR_NOT_CONVERGED and res["iterations"] == K
        np.testing.assert_allclose(x, ref["x"], rtol=0, atol=1e-10 * np.abs(ref["x"]).max(), err_msg=f"K={K}")
        tr = ref["trace"]
        # the first Anderson step with a history: with l >= 2 parallel
        # columns the Cholesky bound cannot hold, so the eigendecomposition
        # ran (the shortcut would report l) and dropped null directions.  How
        # many it drops is not unique: the computed F^T F of parallel columns
        # has l - 1 eigenvalues at the rounding level of its products (about
        # u lambda_max times a summation factor), which straddles the
        # threshold l lambda_max 2^-52, so either side may keep a few of
        # them (they carry no weight in the update: the iterates agree
        # above).  A single column (p = 1, l = 1) is kept by both sides.
        first = next((t for t in range(len(tr)) if min(int(tr[t, 0]), m) >= 1), None)
        if first is None:
            continue   # no extrapolation with a history before the cap
        l_first = min(int(tr[first, 0]), m)
        if l_first >= 2:
            assert 1 <= ranks[first] < l_first, (ranks, tr[:, 4])
            assert 1 <= int(tr[first, 4]) < l_first, tr[:, 4]
        else:
            assert ranks[first] == int(tr[first, 4]) == 1, (ranks, tr[:, 4])
        # the residual after the rank-1 step is at rounding level: the
        # extrapolation is exact for a one-dimensional residual space
        if len(log) > first + 1:
            assert log[first + 1] < 1e-10 * log[first]


SHORT_PERIODIC = [
    ("r6_n456", inputs.Problem(n=(4, 6, 5), h=(0.25, 1 / 6, 0.2), bc=(1, 1, 1), radius=6, shift=0.7)),
    ("r3_n2_1_5_mixed_bc", inputs.Problem(n=(2, 1, 5), h=(0.5, 1.0, 0.2), bc=(1, 1, 0), radius=3, shift=0.2)),
    ("r4_n70_3_9", inputs.Problem(n=(70, 3, 9), h=(1 / 70, 1 / 3, 1 / 9), bc=(1, 1, 1), radius=4, shift=1.5)),
    ("r2_n66_4_3_paired", inputs.Problem(n=(66, 4, 3), h=(1 / 66, 0.25, 1 / 3), bc=(1, 1, 1), radius=2, shift=0.4)),
]


@pytest.mark.parametrize("name,prob", SHORT_PERIODIC, ids=[c[0] for c in SHORT_PERIODIC])
def test_periodic_axis_shorter_than_stencil(name, prob):
    """Periodic axes with n < 2r + 1: the taps wrap modulo n and add up, and
    the Jacobi diagonal includes the taps that land on the point itself
    (operator element by element, iterates at caps, a full solve)."""
    say(f"short periodic {name} n={prob.n}")
    x = inputs.normal(17, 0, prob.size)
    s = aar.Solver([prob], params())
    y = s.apply(to_dev(x)).cpu().numpy()
    s.close()
    ref = oracle.apply(prob, x)
    scale = np.abs(oracle.diagonal(prob)).max() * np.abs(x).max()
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13 * scale)
    b = inputs.normal(5, 0, prob.size)
    for K in (5, 7, 13):
        prm = params(max_iter=K, tol=1e-30)
        xs, res, _, _ = solve_logged(prob, params(max_iter=K, tol=1e-30, flags=aar.AAR_FLAG_RECORD_RESIDUALS), b)
        refx = oracle.aar_solve(prob, b, m=prm.m, p=prm.p, tol=1e-30, max_iter=K)["x"]
        np.testing.assert_allclose(xs, refx, rtol=0, atol=1e-10 * np.abs(refx).max(), err_msg=f"K={K}")
    xs, res, _, _ = solve_logged(prob, params(tol=1e-10, flags=aar.AAR_FLAG_RECORD_RESIDUALS), b)
    assert res["status"] == aar.AAR_OK, res
    assert oracle.relative_residual(prob, b, xs) < 1e-10
