"""GPU parity of the optional constant-mode deflation (AAR_FLAG_DEFLATE_CONSTANT,
not part of the paper's method) against the oracle's own deflation step.

In FP64 mode the solver applies the step once, x0 <- x0 + mean(b - A x0)/sigma,
and then runs the plain AAR iteration from that start; the oracle takes the
same step (oracle.deflate_constant, pinned on the CPU) and runs its AAR from
the result.  Compared: iterates at caps inside and after a cycle (single
system), and for a batch of shifted periodic Helmholtz systems with small
shifts (the near-null constant mode) the iteration counts, the first residuals
r_k and the answers, system by system.
"""
import numpy as np
import pytest

import oracle
from paper_1606_08740_amd import aar, inputs
from tests.gpu_util import gpu_solve, rel_err, say, to_dev

pytestmark = pytest.mark.gpu


def test_fp64_deflated_iterates_match_oracle():
    prob = inputs.periodic_problem(24, 4, shift=0.3)
    b = inputs.normal(12, 0, prob.size) + 0.5
    x0 = oracle.deflate_constant(prob, b)
    p = 6
    for K in (p - 1, p + 1, 2 * p + 3):
        prm = inputs.Params(tol=1e-30, max_iter=K, precision=0, flags=aar.AAR_FLAG_DEFLATE_CONSTANT)
        say(f"deflated iterates K={K}")
        x, res, _ = gpu_solve(prob, prm, b)
        assert res["status"] == aar.AAR_NOT_CONVERGED and res["iterations"] == K
        ref = oracle.aar_solve(prob, b, x0=x0, m=prm.m, p=p, tol=1e-30, max_iter=K)["x"]
        np.testing.assert_allclose(x, ref, rtol=0, atol=1e-10 * np.abs(ref).max(), err_msg=f"K={K}")


def test_batched_deflated_fp64_matches_oracle():
    sizes = [24, 40, 16, 33, 21]
    shifts = [0.02, 0.05, 0.0118, 0.3, 7.0]
    probs = [inputs.periodic_problem(n, 4, shift=s) for n, s in zip(sizes, shifts)]
    bs = [inputs.normal(99 + i, 0, p.size) for i, p in enumerate(probs)]
    prm = inputs.Params(tol=1e-10, precision=0,
                        flags=aar.AAR_FLAG_DEFLATE_CONSTANT | aar.AAR_FLAG_RECORD_RESIDUALS)
    say("batched deflated FP64 vs oracle")
    s = aar.Solver(probs, prm)
    bt = to_dev(np.concatenate(bs))
    xt = to_dev(np.zeros(sum(p.size for p in probs)))
    res = s.solve_batched(bt, xt)
    xs = xt.cpu().numpy()
    logs = [s.residual_log(i) for i in range(len(probs))]
    offs = s.offsets.copy()
    s.close()
    for i, (pr, bi) in enumerate(zip(probs, bs)):
        xi = xs[offs[i]: offs[i + 1]]
        ref = oracle.aar_solve(pr, bi, x0=oracle.deflate_constant(pr, bi), m=prm.m, p=prm.p, tol=prm.tol,
                               trace_cap=100000)
        assert res[i]["status"] == aar.AAR_OK and ref["status"] == oracle.OK, (i, res[i])
        assert oracle.relative_residual(pr, bi, xi) < prm.tol
        # same iteration up to rounding order: within one cycle
        assert abs(res[i]["iterations"] - ref["iterations"]) <= prm.p, (i, res[i], ref["iterations"])
        # the first Anderson-step residuals follow the oracle's trace closely
        np.testing.assert_allclose(logs[i][:3], ref["trace"][:3, 1], rtol=1e-8, err_msg=f"system {i}")
        assert rel_err(xi, ref["x"]) < 1e-7


def test_batched_plain_fp64_converges_without_deflation():
    """The paper's method itself (no deflation) on the same small shifts:
    FP64 converges, matching the oracle's plain AAR within a cycle."""
    sizes = [24, 16, 33]
    shifts = [0.02, 0.0118, 0.3]
    probs = [inputs.periodic_problem(n, 4, shift=s) for n, s in zip(sizes, shifts)]
    bs = [inputs.normal(199 + i, 0, p.size) for i, p in enumerate(probs)]
    prm = inputs.Params(tol=1e-10, precision=0, flags=aar.AAR_FLAG_RECORD_RESIDUALS)
    say("batched plain FP64 small shifts")
    s = aar.Solver(probs, prm)
    bt = to_dev(np.concatenate(bs))
    xt = to_dev(np.zeros(sum(p.size for p in probs)))
    res = s.solve_batched(bt, xt)
    xs = xt.cpu().numpy()
    logs = [s.residual_log(i) for i in range(len(probs))]
    offs = s.offsets.copy()
    s.close()
    for i, (pr, bi) in enumerate(zip(probs, bs)):
        xi = xs[offs[i]: offs[i + 1]]
        ref = oracle.aar_solve(pr, bi, m=prm.m, p=prm.p, tol=prm.tol, trace_cap=100000)
        assert res[i]["status"] == aar.AAR_OK and ref["status"] == oracle.OK, (i, res[i])
        assert oracle.relative_residual(pr, bi, xi) < prm.tol
        assert abs(res[i]["iterations"] - ref["iterations"]) <= max(prm.p, 0.05 * ref["iterations"]), \
            (i, res[i], ref["iterations"])
        np.testing.assert_allclose(logs[i][:3], ref["trace"][:3, 1], rtol=1e-8, err_msg=f"system {i}")
