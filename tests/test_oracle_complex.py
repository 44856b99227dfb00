"""Pins of the oracle's complex-valued AAR (Sec. 2, Eq. 1 over C, Eq. 3 with
complex omega, beta and the conjugate transpose; the periodic Helmholtz
problem of Sec. 3.2, Eq. 7), against what the mathematics fixes:

  * the complex operator equals an independently assembled dense matrix
    (Kronecker products plus i s I) and has the closed-form eigenvalues on
    Fourier modes;
  * with every imaginary part zero it reproduces the real oracle;
  * the solution equals a dense complex LU solve within 10 kappa tol (complex
    omega and beta included, and the indefinite Helmholtz shift of Eq. 7);
  * with complete history and p = 1 the least-squares residuals equal the
    left-preconditioned GMRES residuals (complex Arnoldi, textbook);
  * a Fourier-mode right-hand side makes every history column parallel: the
    Hermitian pseudoinverse truncates and the first extrapolation is exact.
A dropped conjugate, a wrong sign of the imaginary shift, a real-only
pseudoinverse or a transposed product fails one of them.
"""
import numpy as np
import pytest

import oracle
from paper_1606_08740_amd import inputs
from tests.test_oracle_stencil import dense_operator


def _cnormal(seed, n):
    return inputs.normal(seed, 0, n) + 1j * inputs.normal(seed, 1, n)


def test_complex_apply_matches_dense():
    prob = inputs.Problem(n=(5, 4, 6), h=(0.2, 0.25, 1 / 6), bc=(1, 0, 1), radius=3, diffusion=0.3, shift=-0.4)
    x = _cnormal(3, prob.size)
    A = dense_operator(prob) + 1j * 0.7 * np.eye(prob.size)
    np.testing.assert_allclose(oracle.apply_complex(prob, 0.7, x), A @ x, rtol=0, atol=1e-12 * np.abs(A).max())


def test_complex_apply_fourier_eigenvalue():
    n, r, s_im = 8, 3, -0.07
    prob = inputs.Problem(n=(n, n, n), h=(1 / n,) * 3, bc=(1, 1, 1), radius=r, diffusion=1 / (4 * np.pi),
                          shift=-0.13)
    k = (1, 2, 3)
    g = np.arange(n)
    phase = np.exp(2j * np.pi * (k[0] * g[None, None, :] + k[1] * g[None, :, None] + k[2] * g[:, None, None]) / n)
    u = phase.ravel()
    w = oracle.fd_weights(r)
    lam = prob.shift + 1j * s_im
    for ax in range(3):
        th = 2 * np.pi * k[ax] / n
        lam += -prob.diffusion * n ** 2 * (w[0] + 2 * sum(w[s] * np.cos(s * th) for s in range(1, r + 1)))
    np.testing.assert_allclose(oracle.apply_complex(prob, s_im, u), lam * u, rtol=0, atol=1e-11 * abs(lam))


def test_real_data_reproduces_real_oracle():
    prob = inputs.periodic_problem(10, 3, shift=0.8)
    b = inputs.normal(4, 0, prob.size)
    for K in (5, 13, 40):
        c = oracle.aar_solve_complex(prob, b, 0.0, m=7, p=6, tol=1e-30, max_iter=K)["x"]
        r = oracle.aar_solve(prob, b, m=7, p=6, tol=1e-30, max_iter=K)["x"]
        assert np.abs(c.imag).max() == 0.0
        np.testing.assert_allclose(c.real, r, rtol=0, atol=1e-12 * np.abs(r).max())


LU_CASES = [
    ("ofdft_helmholtz_r3", lambda: inputs.ofdft_helmholtz(7, tol=1e-12), 0.6, 0.6),
    ("complex_relaxation", lambda: inputs.ofdft_helmholtz(6, tol=1e-12), 0.6 + 0.2j, 0.5 - 0.1j),
    ("dirichlet_shifted", lambda: (inputs.Problem(n=(5, 4, 3), h=(1 / 6, 1 / 5, 1 / 4), bc=(0, 0, 0), radius=1,
                                                  shift=2.0), 3.0, _cnormal(9, 60), None), 0.6, 0.6),
]


@pytest.mark.parametrize("name,make,omega,beta", LU_CASES, ids=[c[0] for c in LU_CASES])
def test_complex_solution_matches_dense_lu(name, make, omega, beta):
    prob, s_im, b, _ = make()
    tol = 1e-12
    out = oracle.aar_solve_complex(prob, b, s_im, omega=omega, beta=beta, m=7, p=6, tol=tol)
    assert out["status"] == oracle.OK
    A = dense_operator(prob) + 1j * s_im * np.eye(prob.size)
    x_lu = np.linalg.solve(A, b)
    kappa = np.linalg.cond(A)
    err = np.linalg.norm(out["x"] - x_lu) / np.linalg.norm(x_lu)
    assert err <= 10 * kappa * tol
    assert oracle.relative_residual_complex(prob, s_im, b, out["x"]) == pytest.approx(out["relres"], rel=1e-6)


def complex_gmres_residuals(Mi_A, r0, K):
    """Residual norms of GMRES on the left-preconditioned complex operator:
    Arnoldi with modified Gram-Schmidt (conjugated inner products) and a dense
    least-squares solve of the Hessenberg system, steps 0..K."""
    N = r0.size
    Q = np.zeros((N, K + 1), dtype=complex)
    H = np.zeros((K + 1, K), dtype=complex)
    beta0 = np.linalg.norm(r0)
    Q[:, 0] = r0 / beta0
    res = [beta0]
    for j in range(K):
        w = Mi_A @ Q[:, j]
        for i in range(j + 1):
            H[i, j] = np.vdot(Q[:, i], w)
            w = w - H[i, j] * Q[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        Q[:, j + 1] = w / H[j + 1, j]
        e1 = np.zeros(j + 2, dtype=complex)
        e1[0] = beta0
        y = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)[0]
        res.append(np.linalg.norm(e1 - H[: j + 2, : j + 1] @ y))
    return np.array(res)


def test_complete_history_matches_complex_gmres():
    prob, s_im, _, _ = inputs.ofdft_helmholtz(6)
    b = _cnormal(12, prob.size)
    K = 14
    out = oracle.aar_solve_complex(prob, b, s_im, omega=0.6 + 0.1j, beta=0.6, m=K + 1, p=1, tol=1e-30,
                                   max_iter=K + 1, trace_cap=100)
    A = dense_operator(prob) + 1j * s_im * np.eye(prob.size)
    d = np.diag(A)
    g = complex_gmres_residuals(A / d[:, None], b / d, K)
    tr = out["trace"]
    # at step k (k >= 1 columns) the least-squares residual ||f_k - F_k gamma||
    # equals GMRES's residual after k steps
    for t in range(1, K + 1):
        assert tr[t, 3] == pytest.approx(g[t], rel=1e-7, abs=1e-13 * g[0]), (t, tr[t, 3], g[t])


def test_fourier_mode_rank_one_and_exact_step():
    n = 8
    prob = inputs.Problem(n=(n, n, n), h=(1 / n,) * 3, bc=(1, 1, 1), radius=3, diffusion=1 / (4 * np.pi),
                          shift=-0.13)
    s_im = -0.07
    g = np.arange(n)
    b = np.exp(2j * np.pi * (g[None, None, :] + 2 * g[None, :, None] + g[:, None, None]) / n).ravel()
    out = oracle.aar_solve_complex(prob, b, s_im, m=7, p=6, tol=1e-30, max_iter=12, trace_cap=10)
    tr = out["trace"]
    # five parallel columns: the pseudoinverse truncates (how many rounding-level
    # eigenvalues of the computed F^H F clear the threshold is not unique)
    assert 1 <= int(tr[0, 4]) < 5
    assert tr[1, 1] < 1e-12 * tr[0, 1]        # the extrapolation solved the one-mode system
    lam = oracle.apply_complex(prob, s_im, b)[0] / b[0]
    np.testing.assert_allclose(out["x"], b / lam, rtol=0, atol=1e-12 * abs(1 / lam))
