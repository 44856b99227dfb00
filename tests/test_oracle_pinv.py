"""Pins of the oracle's small least-squares solve gamma = pinv(F^T F) F^T f.

The Anderson step (Eq. 3) needs (F^T F)^{-1} F^T f, evaluated with the
Moore-Penrose pseudoinverse because F^T F is ill-conditioned (Sec. 3.2).
Pinned by exact rational arithmetic on integer-valued data, by the
minimum-norm solution of a rank-deficient case derived by hand, and by the
closed-form spectrum of a tridiagonal Toeplitz matrix for the eigen-solver.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1606_08740_amd import inputs


def exact_normal_solve(F, f):
    """Solve (F^T F) g = F^T f exactly over the rationals (full column rank)."""
    F = [[Fraction(int(v)) for v in row] for row in F]
    f = [Fraction(int(v)) for v in f]
    m = len(F[0])
    G = [[sum(F[i][a] * F[i][b] for i in range(len(F))) for b in range(m)] for a in range(m)]
    c = [sum(F[i][a] * f[i] for i in range(len(F))) for a in range(m)]
    M = [row[:] + [c[a]] for a, row in enumerate(G)]
    for col in range(m):
        piv = next(i for i in range(col, m) if M[i][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for i in range(m):
            if i != col:
                fac = M[i][col] / M[col][col]
                M[i] = [x - fac * y for x, y in zip(M[i], M[col])]
    return [M[a][m] / M[a][a] for a in range(m)]


def integer_data(seed, N, m):
    u = inputs.uniform(seed, 0, N * m + N)
    vals = np.floor(u * 11) - 5          # integers in [-5, 5]
    return vals[: N * m].reshape(N, m), vals[N * m:]


@pytest.mark.parametrize("seed,N,m", [(1, 12, 3), (2, 12, 3), (3, 20, 5), (4, 30, 7)])
def test_pinv_solve_exact_rational(seed, N, m):
    F, f = integer_data(seed, N, m)
    if np.linalg.matrix_rank(F) < m:
        pytest.skip("drawn F is rank deficient")
    exact = exact_normal_solve(F, f)
    g, rank = oracle.pinv_solve(F.T @ F, F.T @ f)
    assert rank == m
    np.testing.assert_allclose(g, [float(v) for v in exact], rtol=1e-12, atol=1e-13)


def test_pinv_solve_rank_deficient_min_norm():
    """F = [a, a, b]: the minimum-norm minimizer splits the weight of the
    repeated column evenly: gamma = (t/2, t/2, u) with (t, u) the exact
    least-squares solution for [a, b]."""
    F2, f = integer_data(7, 15, 2)
    t, u = exact_normal_solve(F2, f)
    F = np.column_stack([F2[:, 0], F2[:, 0], F2[:, 1]])
    g, rank = oracle.pinv_solve(F.T @ F, F.T @ f)
    assert rank == 2
    np.testing.assert_allclose(g, [float(t) / 2, float(t) / 2, float(u)], rtol=1e-12, atol=1e-12)


def test_pinv_zero_and_empty():
    g, rank = oracle.pinv_solve(np.zeros((3, 3)), np.zeros(3))
    assert rank == 0 and (g == 0).all()
    g, rank = oracle.pinv_solve(np.zeros((0, 0)), np.zeros(0))
    assert rank == 0 and g.shape == (0,)


def test_pinv_threshold_drops_noise_direction():
    """Eigenvalues below l * lambda_max * 2^-52 are dropped."""
    G = np.diag([1.0, 1e-20])
    g, rank = oracle.pinv_solve(G, np.array([2.0, 3.0]))
    assert rank == 1
    np.testing.assert_allclose(g, [2.0, 0.0])
    G = np.diag([1.0, 1e-14])
    g, rank = oracle.pinv_solve(G, np.array([2.0, 3e-14]))
    assert rank == 2
    np.testing.assert_allclose(g, [2.0, 3.0], rtol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 5, 10, 16])
def test_jacobi_eigen_tridiagonal_toeplitz(n):
    """tridiag(-1, 2, -1) has eigenvalues 2 - 2 cos(k pi / (n+1))."""
    S = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    lam, V = oracle.jacobi_eigen(S)
    exact = np.sort(2 - 2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    np.testing.assert_allclose(np.sort(lam), exact, atol=1e-14)
    np.testing.assert_allclose(V.T @ V, np.eye(n), atol=1e-14)
    np.testing.assert_allclose(S @ V, V * lam[None, :], atol=1e-13)
