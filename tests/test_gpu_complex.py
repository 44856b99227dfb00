"""GPU parity of the complex-valued AAR (aar_create_complex) against the
oracle's complex AAR (Sec. 2 over C: complex omega and beta, the conjugate
transpose in Eq. 3; the periodic Helmholtz problem of Sec. 3.2, Eq. 7),
through the C ABI:
  * the operator A = A_r + i s I element by element (ragged tiles, both
    boundary rules, several radii);
  * iterates at caps inside and after cycles (complex omega and beta, p = 1,
    history lengths up to 8), element by element;
  * full solves of the OF-DFT Helmholtz workload (the paper's P and Q,
    sixth-order periodic FD): residual by the oracle's operator, iteration
    count, answer and the first Anderson-step residuals;
  * a Fourier-mode right-hand side (parallel history columns): the Hermitian
    pseudoinverse truncates and the extrapolation is exact;
  * every tile shape the creation-time timing of the complex sweep can pick,
    forced through a tile file: operator and iterates.
"""
import numpy as np
import pytest

import oracle
from paper_1606_08740_amd import aar, inputs
from tests.gpu_util import params, say

pytestmark = pytest.mark.gpu


def to_dev_c(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.complex128), device="cuda:0")


def cnormal(seed, n):
    return inputs.normal(seed, 0, n) + 1j * inputs.normal(seed, 1, n)


def csolve(prob, prm, s_im, b, omega=None, beta=None):
    import torch
    s = aar.ComplexSolver(prob, prm, s_im, omega=omega, beta=beta)
    bt = to_dev_c(b)
    xt = torch.zeros_like(bt)
    res = s.solve(bt, xt)
    torch.cuda.synchronize()
    log = s.residual_log() if prm.flags & aar.AAR_FLAG_RECORD_RESIDUALS else None
    ranks = s.rank_log() if prm.flags & aar.AAR_FLAG_RECORD_RESIDUALS else None
    out = xt.cpu().numpy()
    s.close()
    return out, res, log, ranks


APPLY_CASES = [
    ("periodic_r3_ragged", inputs.Problem(n=(70, 17, 21), h=(0.1, 0.2, 0.15), bc=(1, 1, 1), radius=3,
                                          diffusion=1 / (4 * np.pi), shift=-0.135), -0.07),
    ("dirichlet_r1", inputs.Problem(n=(33, 20, 9), h=(0.03, 0.05, 0.1), bc=(0, 0, 0), radius=1, shift=0.4), 1.5),
    ("mixed_bc_r6", inputs.Problem(n=(66, 15, 30), h=(0.02, 0.07, 0.03), bc=(1, 0, 1), radius=6), 0.3),
]


@pytest.mark.parametrize("name,prob,s_im", APPLY_CASES, ids=[c[0] for c in APPLY_CASES])
def test_complex_apply_matches_oracle(name, prob, s_im):
    say(f"complex apply {name}")
    x = cnormal(7, prob.size)
    s = aar.ComplexSolver(prob, params(), s_im)
    y = s.apply(to_dev_c(x)).cpu().numpy()
    s.close()
    ref = oracle.apply_complex(prob, s_im, x)
    scale = (np.abs(oracle.diagonal(prob)).max() + abs(s_im)) * np.abs(x).max()
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13 * scale)


ITER_CASES = [
    ("ofdft_r3", lambda: inputs.ofdft_helmholtz(20)[:2], dict(m=7, p=6), 0.6, 0.6),
    ("complex_relaxation", lambda: inputs.ofdft_helmholtz(18)[:2], dict(m=5, p=4), 0.6 + 0.2j, 0.5 - 0.1j),
    ("p1_m8", lambda: (inputs.Problem(n=(24, 19, 13), h=(0.05, 0.06, 0.08), bc=(0, 1, 0), radius=2, shift=0.3),
                       0.9), dict(m=8, p=1), 0.6, 0.6),
    ("m3_dirichlet", lambda: (inputs.Problem(n=(30, 14, 11), h=(0.03, 0.07, 0.09), bc=(0, 0, 0), radius=1,
                                             shift=1.0), -2.0), dict(m=3, p=5), 0.6, 0.6),
]


@pytest.mark.parametrize("force", [0, aar.AAR_FLAG_FORCE_PINV], ids=["auto", "forced_pinv"])
@pytest.mark.parametrize("name,make,kw,omega,beta", ITER_CASES, ids=[c[0] for c in ITER_CASES])
def test_complex_iterates_match_oracle(name, make, kw, omega, beta, force):
    """Both branches of the m x m solve: the Cholesky solve of the real form
    (taken when a bound proves it equals the pseudoinverse) and, forced, the
    Jacobi eigendecomposition."""
    prob, s_im = make()
    b = cnormal(5, prob.size)
    p = kw["p"]
    for K in sorted({1, max(p - 1, 1), p, p + 1, 3 * p + 2}):
        say(f"complex iterates {name} K={K} force={force}")
        x, res, _, _ = csolve(prob, params(max_iter=K, tol=1e-30, flags=force, **kw), s_im, b, omega, beta)
        ref = oracle.aar_solve_complex(prob, b, s_im, omega=omega, beta=beta, m=kw["m"], p=p, tol=1e-30,
                                       max_iter=K)
        assert res["status"] == aar.AAR_NOT_CONVERGED and res["iterations"] == K, res
        np.testing.assert_allclose(x, ref["x"], rtol=0, atol=1e-10 * np.abs(ref["x"]).max(), err_msg=f"K={K}")


@pytest.mark.parametrize("n", [24, 36])
def test_ofdft_helmholtz_full_solve(n):
    prob, s_im, b, prm = inputs.ofdft_helmholtz(n)
    prm.flags = aar.AAR_FLAG_RECORD_RESIDUALS
    say(f"complex OF-DFT Helmholtz n={n}")
    x, res, log, ranks = csolve(prob, prm, s_im, b)
    ref = oracle.aar_solve_complex(prob, b, s_im, m=prm.m, p=prm.p, tol=prm.tol, trace_cap=100000)
    assert res["status"] == aar.AAR_OK and ref["status"] == oracle.OK, res
    rr = oracle.relative_residual_complex(prob, s_im, b, x)
    assert rr < prm.tol
    assert rr == pytest.approx(res["rel_residual"], rel=1e-6)
    assert res["iterations"] % prm.p == 0
    assert abs(res["iterations"] - ref["iterations"]) <= max(prm.p, 0.1 * ref["iterations"])
    # Anderson-step residuals: rounding differences are amplified by each
    # solve with F^H F (cond up to ~1e11 here); step t is compared within 1000
    # u times the summed condition numbers of the solves before it, while that
    # stays below 1e-6
    tr = ref["trace"]
    sens = 1.1e-16 * np.cumsum(np.concatenate([[1.0], tr[:-1, 5]]))
    checked = 0
    for t in range(min(len(tr), len(log))):
        if sens[t] > 1e-6:
            break
        assert log[t] == pytest.approx(tr[t, 1], rel=max(1e-10, 1000 * sens[t])), (t, log[t], tr[t, 1])
        checked += 1
    assert checked >= 1
    assert np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"]) < 1e-6


def test_fourier_mode_truncates_and_is_exact():
    n = 16
    prob = inputs.Problem(n=(n, n, n), h=(1 / n,) * 3, bc=(1, 1, 1), radius=3, diffusion=1 / (4 * np.pi),
                          shift=-0.13)
    s_im = -0.07
    g = np.arange(n)
    b = np.exp(2j * np.pi * (g[None, None, :] + 2 * g[None, :, None] + g[:, None, None]) / n).ravel()
    say("complex Fourier mode")
    x, res, log, ranks = csolve(prob, params(max_iter=12, tol=1e-30, flags=aar.AAR_FLAG_RECORD_RESIDUALS), s_im, b)
    assert 1 <= ranks[0] < 5, ranks
    assert log[1] < 1e-12 * log[0]
    lam = oracle.apply_complex(prob, s_im, b)[0] / b[0]
    np.testing.assert_allclose(x, b / lam, rtol=0, atol=1e-11 * abs(1 / lam))


TILE_CASES = [(1, 2, 0), (1, 4, 2), (2, 2, 3), (1, 6, 1), (2, 32, 0)]


@pytest.mark.parametrize("shape", TILE_CASES, ids=[f"ry{s[0]}_cz{s[1]}_order{s[2]}" for s in TILE_CASES])
def test_complex_tile_shapes_match_oracle(shape, tmp_path, monkeypatch):
    """The complex sweep's tile is timed at creation unless the tile file
    lists the grid (precision field 2); every shape the timing can pick
    (rows per thread, short z chunks with a ragged last one, tile numbering
    and z direction) gives the oracle's operator and iterates."""
    ry, cz, order = shape
    prob = inputs.Problem(n=(70, 13, 23), h=(0.1, 0.2, 0.15), bc=(1, 1, 1), radius=3, diffusion=1 / (4 * np.pi),
                          shift=-0.135)
    s_im = -0.07
    tile = tmp_path / "tiles.txt"
    tile.write_text(f"2 {prob.radius} 0 {prob.n[0]} {prob.n[1]} {prob.n[2]} {ry} {cz} {order} 0 0\n")
    monkeypatch.setenv("AAR_TUNE_CACHE", str(tile))
    say(f"complex tile shape {shape} n={prob.n}")
    x = cnormal(21, prob.size)
    s = aar.ComplexSolver(prob, params(), s_im)
    y = s.apply(to_dev_c(x)).cpu().numpy()
    s.close()
    ref = oracle.apply_complex(prob, s_im, x)
    scale = (np.abs(oracle.diagonal(prob)).max() + abs(s_im)) * np.abs(x).max()
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13 * scale)
    b = cnormal(5, prob.size)
    for K in (5, 7, 13):
        xs, res, _, _ = csolve(prob, params(max_iter=K, tol=1e-30, m=7, p=6), s_im, b, 0.6, 0.6)
        refx = oracle.aar_solve_complex(prob, b, s_im, omega=0.6, beta=0.6, m=7, p=6, tol=1e-30, max_iter=K)["x"]
        assert res["iterations"] == K
        np.testing.assert_allclose(xs, refx, rtol=0, atol=1e-10 * np.abs(refx).max(), err_msg=f"K={K}")
