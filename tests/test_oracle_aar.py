"""Pins of the oracle's AAR iteration (Eqs. 2-6) against what the paper and
the mathematics fix:

  * p -> infinity is the weighted Jacobi / Richardson iteration (Sec. 2): on
    an eigenmode right-hand side its iterates have a closed form;
  * the converged answer agrees with a dense LU solve on tiny grids
    (bordered system for the singular periodic Poisson problem);
  * with complete history the Anderson step minimizes the preconditioned
    residual over the Krylov space, so the extrapolated residual norms equal
    those of left-preconditioned GMRES (Sec. 2, AAR <-> AR <-> GMRES), for
    p = 1 (AR) and p > 1 alike;
  * with finite history each update is the minimizer over the last m
    iterate differences only (Eqs. 3-5), checked against iterates with a
    dense operator and a library least-squares solve;
  * invariants: convergence is tested only at Anderson steps, so iteration
    counts are multiples of p (Sec. 2); the returned iterate's residual is
    the reported one; the extrapolated residual never exceeds ||f_k||;
  * manufactured solutions, power-of-two scale invariance, axis symmetry,
    and the degenerate inputs (b = 0, NaN, iteration cap).
"""
import numpy as np
import pytest

import oracle
from paper_1606_08740_amd import inputs
from tests.test_oracle_stencil import dense_operator


def cd_problem(n=6, seed=4, bc=0):
    v = inputs.convection_field(n, seed, peclet=0.9)
    return inputs.Problem(n=(n, n, n), h=(1 / (n + 1),) * 3, bc=(bc,) * 3, radius=1, velocity=v)


# ---------------------------------------------------------------------------
# Richardson limit (p -> infinity)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("omega", [0.6, 1.0])
def test_richardson_limit_closed_form(omega):
    """x_n = [1 - (1 - omega lambda / d)^n] phi / lambda for A phi = lambda phi,
    constant diagonal d, x_0 = 0, no Anderson step (p > n)."""
    n = (9, 7, 8)
    h = tuple(1.0 / (v + 1) for v in n)
    prob = inputs.Problem(n=n, h=h, bc=(0, 0, 0), radius=1)
    a, b, c = 2, 3, 1
    xs = [np.sin(q * np.pi * (np.arange(nn) + 1) * hh) for q, nn, hh in zip((a, b, c), n, h)]
    phi = (xs[2][:, None, None] * xs[1][None, :, None] * xs[0][None, None, :]).reshape(-1)
    lam = sum(4.0 / hh ** 2 * np.sin(q * np.pi * hh / 2) ** 2 for q, hh in zip((a, b, c), h))
    d = sum(2.0 / hh ** 2 for hh in h)
    for steps in [1, 2, 7, 25]:
        out = oracle.aar_solve(prob, phi, m=3, p=steps + 1, tol=1e-30, max_iter=steps, omega=omega)
        assert out["status"] == oracle.NOT_CONVERGED and out["iterations"] == steps
        expect = (1 - (1 - omega * lam / d) ** steps) * phi / lam
        np.testing.assert_allclose(out["x"], expect, rtol=0, atol=1e-13 * np.abs(phi / lam).max())


def test_richardson_limit_matches_jacobi_sweeps():
    """Richardson with M = D on a random rhs is the weighted Jacobi sweep
    x <- x + omega D^{-1}(b - A x) with A, D from the dense operator."""
    prob = cd_problem(5)
    A = dense_operator(prob)
    D = np.diag(A)
    b = inputs.normal(5, 0, prob.size)
    x = np.zeros(prob.size)
    for _ in range(9):
        x = x + 0.6 * (b - A @ x) / D
    out = oracle.aar_solve(prob, b, m=4, p=100, tol=1e-30, max_iter=9)
    np.testing.assert_allclose(out["x"], x, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------
# Dense LU
# ---------------------------------------------------------------------------
def lu_reference(prob, b, singular=False):
    A = dense_operator(prob)
    if not singular:
        return np.linalg.solve(A, b), np.linalg.cond(A)
    N = prob.size
    B = np.zeros((N + 1, N + 1))
    B[:N, :N] = A
    B[:N, N] = 1.0
    B[N, :N] = 1.0
    sol = np.linalg.solve(B, np.concatenate([b, [0.0]]))
    ev = np.sort(np.abs(np.linalg.eigvals(A)))
    return sol[:N], ev[-1] / ev[1]


LU_CASES = [
    ("dirichlet_r1", lambda: inputs.Problem(n=(5, 4, 3), h=(1 / 6, 1 / 5, 1 / 4), bc=(0, 0, 0), radius=1), False),
    ("periodic_poisson_r3", lambda: inputs.periodic_problem(6, 3), True),
    ("periodic_helmholtz_r4", lambda: inputs.periodic_problem(7, 4, shift=3.0), False),
    ("upwind_cd", lambda: cd_problem(6), False),
    ("periodic_r6_wrap", lambda: inputs.Problem(n=(8, 5, 6), h=(1 / 8, 1 / 5, 1 / 6), bc=(1, 1, 1),
                                                radius=6, shift=0.5), False),
]


@pytest.mark.parametrize("name,make,singular", LU_CASES, ids=[c[0] for c in LU_CASES])
def test_solution_matches_dense_lu(name, make, singular):
    prob = make()
    b = inputs.normal(21, 0, prob.size)
    if singular:
        b -= b.mean()
    tol = 1e-12
    out = oracle.aar_solve(prob, b, tol=tol, m=7, p=6)
    assert out["status"] == oracle.OK
    x_lu, kappa = lu_reference(prob, b, singular)
    x = out["x"] - out["x"].mean() if singular else out["x"]
    err = np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu)
    assert err <= 10 * kappa * tol


# ---------------------------------------------------------------------------
# GMRES equivalence with complete history
# ---------------------------------------------------------------------------
def gmres_residuals(Mi_A, r0, K):
    """Residual norms ||r_k|| of GMRES on the left-preconditioned operator,
    k = 0..K, by Arnoldi with modified Gram-Schmidt and a dense least-squares
    solve of the Hessenberg system (textbook GMRES)."""
    N = r0.size
    Q = np.zeros((N, K + 1))
    H = np.zeros((K + 1, K))
    beta0 = np.linalg.norm(r0)
    Q[:, 0] = r0 / beta0
    res = [beta0]
    for j in range(K):
        w = Mi_A @ Q[:, j]
        for i in range(j + 1):
            H[i, j] = Q[:, i] @ w
            w = w - H[i, j] * Q[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        Q[:, j + 1] = w / H[j + 1, j]
        e1 = np.zeros(j + 2)
        e1[0] = beta0
        y = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)[0]
        res.append(np.linalg.norm(e1 - H[: j + 2, : j + 1] @ y))
    return np.array(res)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_complete_history_matches_gmres(p):
    """AAR with m >= k minimizes ||M^{-1}(b - A x)|| over x_0 + K_k(M^{-1}A, f_0)
    at each Anderson step k, exactly as GMRES does (nonsymmetric upwind
    operator, Jacobi preconditioner)."""
    prob = cd_problem(6)
    A = dense_operator(prob)
    D = np.diag(A)
    b = inputs.normal(8, 0, prob.size)
    K = 24
    out = oracle.aar_solve(prob, b, m=K + 2, p=p, tol=1e-30, max_iter=K + 1, beta=0.6, omega=0.6,
                           trace_cap=K + 1)
    tr = out["trace"]
    g = gmres_residuals(A / D[:, None], b / D, K)
    ks = tr[:, 0].astype(int)
    got = tr[:, 3]
    ref = g[ks]
    keep = ref > 1e-9 * g[0]
    assert keep.sum() >= 6
    np.testing.assert_allclose(got[keep], ref[keep], rtol=1e-7)


# ---------------------------------------------------------------------------
# Finite history window
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,p", [(3, 2), (4, 3), (5, 1), (2, 4)])
def test_update_minimizes_over_last_m_differences(m, p):
    """Each Anderson update equals x_k + beta f_k - (X_k + beta F_k) gamma with
    X_k, F_k the last min(k, m) iterate / residual differences (Eqs. 3-5) and
    gamma the least-squares minimizer of ||f_k - F_k gamma||; iterates taken
    from the oracle, operator and solver from independent code."""
    prob = cd_problem(5, seed=6)
    A = dense_operator(prob)
    D = np.diag(A)
    b = inputs.normal(9, 0, prob.size)
    beta, omega = 0.7, 0.5
    K = 4 * p + m + 2
    xs = [np.zeros(prob.size)]
    for j in range(1, K + 1):
        o = oracle.aar_solve(prob, b, m=m, p=p, tol=1e-30, max_iter=j, beta=beta, omega=omega)
        xs.append(o["x"])
    fs = [(b - A @ x) / D for x in xs]
    checked = 0
    for k in range(K):
        if (k + 1) % p:
            np.testing.assert_allclose(xs[k + 1], xs[k] + omega * fs[k], rtol=1e-12, atol=1e-15)
            continue
        l = min(k, m)
        X = np.column_stack([xs[i + 1] - xs[i] for i in range(k - l, k)]) if l else np.zeros((prob.size, 0))
        F = np.column_stack([fs[i + 1] - fs[i] for i in range(k - l, k)]) if l else np.zeros((prob.size, 0))
        gam = np.linalg.lstsq(F, fs[k], rcond=None)[0] if l else np.zeros(0)
        pred = xs[k] + beta * fs[k] - (X + beta * F) @ gam
        scale = np.abs(xs[k + 1]).max()
        np.testing.assert_allclose(xs[k + 1], pred, rtol=0, atol=1e-8 * scale)
        checked += 1
    assert checked >= 4


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,p", [(7, 6), (10, 4), (9, 8), (3, 1)])
def test_iterations_multiple_of_p_and_residual_consistent(m, p):
    prob = inputs.dirichlet_poisson_problem(12)
    b = inputs.normal(1, 0, prob.size)
    out = oracle.aar_solve(prob, b, m=m, p=p, tol=1e-9, trace_cap=10000)
    assert out["status"] == oracle.OK
    assert out["iterations"] % p == 0
    tr = out["trace"]
    np.testing.assert_array_equal(tr[:, 0] + 1, np.arange(1, len(tr) + 1) * p)
    assert out["relres"] < 1e-9 and tr[-1, 1] == out["relres"]
    assert (tr[:-1, 1] >= 1e-9).all()
    assert oracle.relative_residual(prob, b, out["x"]) == pytest.approx(out["relres"], rel=1e-6)
    # the extrapolated residual never exceeds the current one (gamma = 0 is admissible)
    assert (tr[:-1, 3] <= tr[:-1, 2] * (1 + 1e-12)).all()


def test_manufactured_solution_within_condition_bound():
    n = 16
    prob = inputs.dirichlet_poisson_problem(n)
    h = prob.h[0]
    lam_min = 3 * 4 / h ** 2 * np.sin(np.pi * h / 2) ** 2
    lam_max = 3 * 4 / h ** 2 * np.sin(n * np.pi * h / 2) ** 2
    kappa = lam_max / lam_min
    xstar = inputs.normal(2, 0, prob.size)
    b = oracle.apply(prob, xstar)
    tol = 1e-10
    out = oracle.aar_solve(prob, b, tol=tol)
    assert out["status"] == oracle.OK
    assert np.linalg.norm(out["x"] - xstar) / np.linalg.norm(xstar) <= kappa * tol


def test_power_of_two_scaling_is_bitwise_invariant():
    """(A, b) -> (4A, 4b) via h -> h/2: every iterate is bitwise identical."""
    p1 = inputs.periodic_problem(10, 4, shift=1.0)
    p2 = inputs.Problem(n=p1.n, h=tuple(v / 2 for v in p1.h), bc=p1.bc, radius=4, shift=4.0)
    b = inputs.normal(3, 0, p1.size)
    for cap in [5, 23, 10 ** 6]:
        o1 = oracle.aar_solve(p1, b, max_iter=cap, tol=1e-10)
        o2 = oracle.aar_solve(p2, 4 * b, max_iter=cap, tol=1e-10)
        assert o1["iterations"] == o2["iterations"]
        np.testing.assert_array_equal(o1["x"], o2["x"])


def test_axis_permutation_symmetry():
    n = 9
    prob = inputs.periodic_problem(n, 3, shift=2.0)
    b = inputs.normal(4, 0, prob.size).reshape(n, n, n)
    o1 = oracle.aar_solve(prob, b.reshape(-1), tol=1e-11)
    o2 = oracle.aar_solve(prob, b.transpose(2, 1, 0).copy().reshape(-1), tol=1e-11)
    np.testing.assert_allclose(o2["x"].reshape(n, n, n), o1["x"].reshape(n, n, n).transpose(2, 1, 0),
                               rtol=0, atol=1e-9 * np.abs(o1["x"]).max())


# ---------------------------------------------------------------------------
# Degenerate inputs
# ---------------------------------------------------------------------------
def test_zero_rhs_returns_zero():
    prob = inputs.dirichlet_poisson_problem(4)
    out = oracle.aar_solve(prob, np.zeros(prob.size), x0=np.ones(prob.size))
    assert out["status"] == oracle.OK and out["iterations"] == 0
    assert (out["x"] == 0).all()


def test_nan_rhs_is_breakdown():
    prob = inputs.dirichlet_poisson_problem(4)
    b = np.ones(prob.size)
    b[5] = np.nan
    out = oracle.aar_solve(prob, b, p=3)
    assert out["status"] == oracle.BREAKDOWN and out["iterations"] == 3


def test_iteration_cap_and_bad_args():
    prob = inputs.dirichlet_poisson_problem(8)
    b = inputs.normal(1, 0, prob.size)
    out = oracle.aar_solve(prob, b, tol=1e-14, max_iter=13)
    assert out["status"] == oracle.NOT_CONVERGED and out["iterations"] == 13
    assert oracle.aar_solve(prob, b, m=0)["status"] == oracle.BAD_ARG
    assert oracle.aar_solve(prob, b, p=0)["status"] == oracle.BAD_ARG
    assert oracle.aar_solve(prob, b, tol=0.0)["status"] == oracle.BAD_ARG


def test_exact_initial_guess_stops_at_first_check():
    prob = inputs.periodic_problem(6, 2, shift=1.0)
    xstar = inputs.normal(6, 0, prob.size)
    b = oracle.apply(prob, xstar)
    out = oracle.aar_solve(prob, b, x0=xstar, p=5, tol=1e-12)
    assert out["status"] == oracle.OK and out["iterations"] == 5
    np.testing.assert_allclose(out["x"], xstar, rtol=0, atol=1e-12 * np.abs(xstar).max())
