"""Pins of the oracle's constant-mode step (the solver's optional deflation;
not part of the paper's method), checked against what the mathematics fixes:

  * A 1 = sigma 1 on an all-periodic grid, so after x' = x + mean(b - A x)/sigma
    the residual b - A x' has zero mean (to rounding);
  * from x = 0 the step is the closed form x' = (mean b / sigma) 1;
  * the AAR solve started from x' reaches the same solution as from 0, within
    the conditioning bound kappa * tol (kappa from the Fourier symbol);
  * a Dirichlet axis or sigma = 0 is refused.
A sign error, a dropped 1/sigma, or a sum instead of a mean fails one of them.
"""
import numpy as np
import pytest

import oracle
from paper_1606_08740_amd import inputs


def _problem(n=(10, 12, 9), r=4, sigma=0.05):
    return inputs.Problem(n=n, h=tuple(1.0 / k for k in n), bc=(1, 1, 1), radius=r, shift=sigma)


@pytest.mark.parametrize("sigma", [0.01, 0.3, 5.0])
def test_deflated_residual_is_mean_free(sigma):
    prob = _problem(sigma=sigma)
    b = inputs.normal(3, 0, prob.size) + 2.0
    x0 = inputs.normal(4, 0, prob.size)
    x = oracle.deflate_constant(prob, b, x0)
    r = b - oracle.apply(prob, x)
    scale = np.abs(b).max() + np.abs(oracle.apply(prob, x0)).max()
    assert abs(r.mean()) <= 1e-13 * scale
    # the step moved x by a constant only
    d = x - x0
    assert np.ptp(d) <= 1e-14 * np.abs(d).max()


def test_step_from_zero_is_closed_form():
    prob = _problem(sigma=0.25)
    b = inputs.normal(5, 0, prob.size) + 1.5
    x = oracle.deflate_constant(prob, b)
    np.testing.assert_allclose(x, np.full(prob.size, b.mean() / 0.25), rtol=1e-14, atol=0)


def test_solution_unchanged_within_condition_bound():
    prob = _problem(n=(8, 8, 8), r=4, sigma=0.2)
    b = inputs.normal(6, 0, prob.size) + 0.7
    tol = 1e-10     # well above the FP64 floor u kappa (kappa ~ 6e3 here)
    plain = oracle.aar_solve(prob, b, tol=tol, max_iter=20000)
    defl = oracle.aar_solve(prob, b, x0=oracle.deflate_constant(prob, b), tol=tol, max_iter=20000)
    assert plain["status"] == defl["status"] == oracle.OK
    # kappa(A) = lambda_max / sigma from the Fourier symbol of the order-2r rule
    w = oracle.fd_weights(4)
    th = 2 * np.pi * np.arange(8) / 8
    sym = -(w[0] + 2 * sum(w[s] * np.cos(s * th) for s in range(1, 5))) * 64.0
    kappa = (3 * sym.max() + prob.shift) / prob.shift
    err = np.linalg.norm(defl["x"] - plain["x"]) / np.linalg.norm(plain["x"])
    assert err <= 10 * kappa * tol
    # the constant component the deflated start carries is the exact one
    assert abs(defl["x"].mean() - b.mean() / prob.shift) <= 10 * kappa * tol * abs(b.mean() / prob.shift)


@pytest.mark.parametrize("change", [dict(bc=(1, 0, 1)), dict(shift=0.0)])
def test_refused_without_constant_eigenvector(change):
    prob = _problem()
    for k, v in change.items():
        setattr(prob, k, v)
    with pytest.raises(ValueError):
        oracle.deflate_constant(prob, np.ones(prob.size))
