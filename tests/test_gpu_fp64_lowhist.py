"""GPU parity of the FP64 iteration with a reduced-precision history ring
(FP32 or bfloat16 columns of F_k, Eqs. 4-5), against the FP64 CPU oracle.

The iterate and the residual of each cycle's first step stay in FP64; the
stored residual history is rounded, which perturbs the Anderson
extrapolation direction but not the fixed point.  With an FP32 ring the
residuals of the cycle's later steps, the Anderson step's
included, follow the residual recursion in FP32 on the ring, which restarts
from the FP64 residual every cycle, so the reported residual matches the
returned x's FP64 residual to ~1e-6 relative.  Parity is therefore on the
answer and on the decision: the oracle's own operator must confirm
||b - A x|| / ||b|| < tol for the returned x, the residual the solver
reported must be that x's residual, and x must match the oracle's solution
within the conditioning bound.  Iteration counts are compared loosely (the
extrapolation path differs from the FP64 one).
"""
import numpy as np
import pytest

import oracle
from paper_1606_08740_amd import aar, inputs
from tests.gpu_util import gpu_solve, mean_free, params, rel_err, say

pytestmark = pytest.mark.gpu

CASES = [
    ("c1_32_dirichlet", lambda: inputs.workload(1, tol=1e-10), False),
    ("periodic_r6_40", lambda: inputs.workload(3, n=40), True),
    ("upwind_24", lambda: inputs.workload(4, n=24), False),
    ("ragged_dirichlet_r3_37x29x23", lambda: inputs.Workload(
        "r", [inputs.Problem(n=(37, 29, 23), h=(0.1, 0.1, 0.1), bc=(0, 0, 0), radius=3)],
        [inputs.normal(21, 0, 37 * 29 * 23)], [None], params(tol=1e-10)), False),
]


@pytest.mark.parametrize("precision", [aar.AAR_FP64_FP32HIST, aar.AAR_FP64_BF16HIST], ids=["fp32hist", "bf16hist"])
@pytest.mark.parametrize("name,make,singular", CASES, ids=[c[0] for c in CASES])
def test_lowhist_reaches_tolerance(name, make, singular, precision):
    w = make()
    prob, b, prm = w.problems[0], w.b[0], w.params
    prm.precision = precision
    prm.flags |= aar.AAR_FLAG_RECORD_RESIDUALS
    say(f"fp64 iterate, history precision {precision}, {name} n={prob.n}")
    x, res, log = gpu_solve(prob, prm, b)
    assert res["status"] == aar.AAR_OK, res
    assert res["outer_steps"] == 0
    assert res["iterations"] % prm.p == 0
    assert len(log) == res["iterations"] // prm.p
    rr = oracle.relative_residual(prob, b, x)
    assert rr < prm.tol
    assert rr == pytest.approx(res["rel_residual"], rel=1e-3, abs=1e-3 * prm.tol)
    ref = oracle.aar_solve(prob, b, m=prm.m, p=prm.p, tol=prm.tol)
    a, r = (mean_free(x), mean_free(ref["x"])) if singular else (x, ref["x"])
    assert rel_err(a, r) < 1e-6
    # rounding the history costs at most a modest number of extra cycles
    assert res["iterations"] <= 1.5 * ref["iterations"] + 4 * prm.p


def test_lowhist_first_cycle_close_to_fp64():
    """Before the first Anderson step the history only feeds Richardson
    increments omega f_j, so the residual of the first Anderson step differs
    from FP64 by the history rounding alone (relative 2^-24 per column for
    FP32, 2^-8 for bfloat16, amplified by the least-squares conditioning)."""
    prob = inputs.dirichlet_poisson_problem(24)
    b = inputs.normal(5, 0, prob.size)
    logs = {}
    for prec in (aar.AAR_FP64, aar.AAR_FP64_FP32HIST, aar.AAR_FP64_BF16HIST):
        prm = params(tol=1e-30, max_iter=2 * 6, m=7, p=6, precision=prec, flags=aar.AAR_FLAG_RECORD_RESIDUALS)
        say(f"first cycles precision {prec}")
        _, res, log = gpu_solve(prob, prm, b)
        assert res["status"] == aar.AAR_NOT_CONVERGED
        logs[prec] = log
    assert logs[aar.AAR_FP64][0] == pytest.approx(logs[aar.AAR_FP64_FP32HIST][0], rel=1e-4)
    assert logs[aar.AAR_FP64][0] == pytest.approx(logs[aar.AAR_FP64_BF16HIST][0], rel=5e-2)


CAP_CASES = [
    ("dirichlet_r1_32", lambda: inputs.dirichlet_poisson_problem(32)),
    ("dirichlet_r1_27_odd", lambda: inputs.dirichlet_poisson_problem(27)),
    ("periodic_r6_30", lambda: inputs.periodic_problem(30, 6, shift=0.5)),
    ("upwind_20", lambda: inputs.workload(4, n=20).problems[0]),
]


@pytest.mark.parametrize("name,make", CAP_CASES, ids=[c[0] for c in CAP_CASES])
def test_fp32hist_iterates_match_oracle(name, make):
    """Iteration caps inside and at the end of a cycle: x_K of the FP64
    iteration over an FP32 ring (the recursion in FP32 on the ring, the
    unfinished cycle's steps added when the run stops) against the oracle's
    FP64 x_K; the difference is the FP32 rounding of the history."""
    prob = make()
    b = inputs.normal(23, 0, prob.size)
    m, p = 7, 6
    for K in (1, p - 1, p, p + 1, 2 * p + 1):
        prm = params(tol=1e-30, max_iter=K, m=m, p=p, precision=aar.AAR_FP64_FP32HIST)
        say(f"fp32hist iterates {name} K={K}")
        x, res, _ = gpu_solve(prob, prm, b)
        assert res["status"] == aar.AAR_NOT_CONVERGED and res["iterations"] == K, (K, res)
        ref = oracle.aar_solve(prob, b, m=m, p=p, tol=1e-30, max_iter=K)["x"]
        np.testing.assert_allclose(x, ref, rtol=0, atol=1e-5 * np.abs(ref).max(), err_msg=f"K={K}")


@pytest.mark.parametrize("precision", [aar.AAR_FP64_FP32HIST, aar.AAR_FP64_BF16HIST], ids=["fp32hist", "bf16hist"])
def test_lowhist_batched_engine(precision):
    """Several systems of uneven sizes and shifts in one call run on the
    batched engine with the narrow history; each answer is checked with the
    oracle's operator and against the same system solved alone."""
    import torch
    probs = [inputs.periodic_problem(n, 4, shift=s) for n, s in [(20, 1.0), (27, 3.0), (33, 0.5), (16, 7.0)]]
    bs = [inputs.normal(30 + i, 0, p.size) for i, p in enumerate(probs)]
    prm = params(tol=1e-10, precision=precision, flags=aar.AAR_FLAG_DEFLATE_CONSTANT)
    say(f"lowhist batched engine precision {precision}")
    s = aar.Solver(probs, prm)
    bt = torch.as_tensor(np.concatenate(bs), device="cuda:0")
    xt = torch.zeros_like(bt)
    res = s.solve_batched(bt, xt)
    torch.cuda.synchronize()
    s.close()
    x = xt.cpu().numpy()
    off = np.concatenate([[0], np.cumsum([p.size for p in probs])])
    for i, p in enumerate(probs):
        assert res[i]["status"] == aar.AAR_OK, (i, res[i])
        xi = x[off[i]:off[i + 1]]
        assert oracle.relative_residual(p, bs[i], xi) < prm.tol
        xs, rs, _ = gpu_solve(p, prm, bs[i])
        assert rs["status"] == aar.AAR_OK
        assert rel_err(xi, xs) < 1e-7
