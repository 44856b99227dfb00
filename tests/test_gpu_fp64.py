"""GPU parity of the FP64 AAR path against the CPU oracle, through the C ABI.

  * the operator (aar_apply) element by element on grids spanning several
    tiles with ragged tails, every radius, both boundary rules, convection;
  * the iterates after K iterations (K inside the first cycles, at and just
    after Anderson steps), element by element: every step of Eqs. 2-6;
  * the residual r_k at every Anderson step of a full solve, the iteration
    count (within one cycle) and the answer;
  * edge cases: b = 0, NaN, history longer than the fast Gram path, p = 1,
    p > m, warm start at the solution.
Tolerances: FP64 rounding differs only in summation order, so iterates
agree to ~1e-12 relative over a few cycles; full solves are compared within
the conditioning bound kappa * tol.
"""
import numpy as np
import pytest

import oracle
from paper_1606_08740_amd import aar, inputs
from tests.gpu_util import gpu_solve, params, rel_err, say, to_dev, mean_free

pytestmark = pytest.mark.gpu


def cd_problem(n, seed=4, bc=0):
    nn = n if isinstance(n, tuple) else (n, n, n)
    v = inputs.convection_field(nn[0], seed) if len(set(nn)) == 1 else \
        inputs.normal(seed, 5, 3 * nn[0] * nn[1] * nn[2]) * 50.0
    h = tuple(1.0 / (k + 1) for k in nn)
    return inputs.Problem(n=nn, h=h, bc=(bc,) * 3, radius=1, velocity=v)


APPLY_CASES = [
    ("dirichlet_r1_ragged", inputs.Problem(n=(70, 37, 41), h=(1 / 71, 1 / 38, 1 / 42), bc=(0, 0, 0), radius=1)),
    ("periodic_r6_ragged", inputs.Problem(n=(67, 29, 33), h=(1 / 67, 1 / 29, 1 / 33), bc=(1, 1, 1), radius=6)),
    ("periodic_r4_shift", inputs.Problem(n=(48, 40, 17), h=(0.02, 0.025, 0.06), bc=(1, 1, 1), radius=4, shift=3.0)),
    ("mixed_bc_r3", inputs.Problem(n=(65, 19, 23), h=(0.01, 0.05, 0.04), bc=(1, 0, 1), radius=3, diffusion=0.7)),
    ("dirichlet_r5_small", inputs.Problem(n=(9, 3, 20), h=(0.1, 0.3, 0.05), bc=(0, 0, 0), radius=5)),
    ("dirichlet_r2", inputs.Problem(n=(130, 9, 5), h=(0.01, 0.1, 0.2), bc=(0, 0, 0), radius=2, shift=0.1)),
    ("upwind_dirichlet", cd_problem((66, 35, 21))),
    ("upwind_periodic", cd_problem((64, 8, 12), bc=1)),
    ("single_point_axis", inputs.Problem(n=(1, 70, 3), h=(1.0, 0.01, 0.3), bc=(0, 1, 0), radius=1)),
]


@pytest.mark.parametrize("name,prob", APPLY_CASES, ids=[c[0] for c in APPLY_CASES])
def test_apply_matches_oracle(name, prob):
    say(f"apply {name} n={prob.n}")
    x = inputs.normal(17, 0, prob.size)
    s = aar.Solver([prob], params())
    y = s.apply(to_dev(x)).cpu().numpy()
    s.close()
    ref = oracle.apply(prob, x)
    scale = np.abs(oracle.diagonal(prob)).max() * np.abs(x).max()
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13 * scale)


ITER_CASES = [
    ("dirichlet_r1", inputs.dirichlet_poisson_problem(20), dict(m=7, p=6)),
    ("periodic_r6", inputs.Problem(n=(26, 25, 27), h=(1 / 26, 1 / 25, 1 / 27), bc=(1, 1, 1), radius=6, shift=0.5),
     dict(m=7, p=6)),
    ("upwind_m10_p4", cd_problem(18), dict(m=10, p=4)),
    ("periodic_r4_p1", inputs.periodic_problem(24, 4, shift=2.0), dict(m=5, p=1)),
    ("dirichlet_p_gt_m", inputs.dirichlet_poisson_problem(17), dict(m=3, p=5)),
    ("long_history_m20", inputs.Problem(n=(70, 9, 11), h=(0.02, 0.1, 0.1), bc=(0, 0, 0), radius=1), dict(m=20, p=2)),
    # the m x m solve runs in registers up to m = 8 and in LDS from m = 9
    ("register_solve_m8", inputs.Problem(n=(30, 22, 17), h=(0.03, 0.04, 0.05), bc=(1, 0, 0), radius=2, shift=0.4),
     dict(m=8, p=3)),
    ("lds_solve_m9", inputs.Problem(n=(30, 22, 17), h=(0.03, 0.04, 0.05), bc=(1, 0, 0), radius=2, shift=0.4),
     dict(m=9, p=3)),
    ("single_column_m1", inputs.dirichlet_poisson_problem(19), dict(m=1, p=1)),
]


@pytest.mark.parametrize("name,prob,kw", ITER_CASES, ids=[c[0] for c in ITER_CASES])
def test_iterates_match_oracle(name, prob, kw):
    b = inputs.normal(5, 0, prob.size)
    p = kw["p"]
    for K in sorted({1, max(p - 1, 1), p, p + 1, 3 * p + 2, 5 * p}):
        say(f"iterates {name} K={K}")
        prm = params(max_iter=K, tol=1e-30, **kw)
        x, res, _ = gpu_solve(prob, prm, b)
        ref = oracle.aar_solve(prob, b, m=kw["m"], p=p, tol=1e-30, max_iter=K)
        assert res["status"] == aar.AAR_NOT_CONVERGED and res["iterations"] == K
        scale = np.abs(ref["x"]).max()
        np.testing.assert_allclose(x, ref["x"], rtol=0, atol=1e-10 * scale, err_msg=f"K={K}")


SOLVE_CASES = [
    ("c1_32_dirichlet_1e-8", lambda: inputs.workload(1), None),
    ("c1_32_dirichlet_1e-10", lambda: inputs.workload(1, tol=1e-10), None),
    ("periodic_r6_40", lambda: inputs.workload(2, n=40), "mean_free"),
    ("upwind_24", lambda: inputs.workload(4, n=24, precision=0), None),
    ("helmholtz_r4_30", lambda: inputs.Workload("h", [inputs.periodic_problem(30, 4, shift=0.7)],
                                                [inputs.normal(9, 0, 27000)], [None], inputs.Params(tol=1e-10)),
     None),
]


@pytest.mark.parametrize("name,make,cmp", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_full_solve_matches_oracle(name, make, cmp):
    w = make()
    prob, b = w.problems[0], w.b[0]
    prm = w.params
    prm.precision = 0
    prm.flags = aar.AAR_FLAG_RECORD_RESIDUALS
    say(f"solve {name} n={prob.n} tol={prm.tol}")
    x, res, log = gpu_solve(prob, prm, b)
    ref = oracle.aar_solve(prob, b, m=prm.m, p=prm.p, tol=prm.tol, trace_cap=100000)
    assert res["status"] == aar.AAR_OK and ref["status"] == oracle.OK
    assert res["iterations"] % prm.p == 0
    # the oracle's own operator confirms the residual
    rr = oracle.relative_residual(prob, b, x)
    assert rr < prm.tol
    assert rr == pytest.approx(res["rel_residual"], rel=1e-6)
    # Anderson-step residuals: the two sides differ only in rounding, which
    # each pseudoinverse solve amplifies by cond(F^T F) (ill-conditioned for
    # smooth right-hand sides, Sec. 2); step t is compared within 1000 u times
    # the summed condition numbers of the solves before it, plus the rounding
    # of ||b - A x|| itself (cancellation, ~u || |A| |x| || / ||b||).
    tr = ref["trace"]
    floor = 1000 * 1.1e-16 * 2 * np.abs(oracle.diagonal(prob)).max() * np.linalg.norm(ref["x"]) / np.linalg.norm(b)
    n = min(len(tr), len(log))
    sens = 1.1e-16 * np.cumsum(np.concatenate([[1.0], tr[:-1, 5]]))[:n]
    checked = 0
    for t in range(n):
        if sens[t] > 1e-6:
            break
        tol_t = max(1e-10, 1000 * sens[t])
        assert abs(log[t] - tr[t, 1]) <= tol_t * tr[t, 1] + floor, (t, log[t], tr[t, 1], tol_t, floor)
        checked += 1
    assert checked >= 1
    if sens[-1] < 1e-6:
        assert abs(res["iterations"] - ref["iterations"]) <= prm.p
    else:
        assert abs(res["iterations"] - ref["iterations"]) <= max(prm.p, 0.1 * ref["iterations"])
    a, r = (mean_free(x), mean_free(ref["x"])) if cmp == "mean_free" else (x, ref["x"])
    assert rel_err(a, r) < 1e-6


def test_zero_rhs():
    prob = inputs.dirichlet_poisson_problem(16)
    say("zero rhs")
    x, res, _ = gpu_solve(prob, params(), np.zeros(prob.size), x0=np.ones(prob.size))
    assert res["status"] == aar.AAR_OK and res["iterations"] == 0
    assert (x == 0).all()


def test_nan_rhs_breakdown():
    prob = inputs.dirichlet_poisson_problem(16)
    b = np.ones(prob.size)
    b[100] = np.nan
    say("nan rhs")
    x, res, _ = gpu_solve(prob, params(p=3), b)
    assert res["status"] == aar.AAR_BREAKDOWN and res["iterations"] == 3


def test_warm_start_at_solution():
    prob = inputs.periodic_problem(20, 3, shift=1.0)
    xstar = inputs.normal(6, 0, prob.size)
    b = oracle.apply(prob, xstar)
    say("warm start")
    x, res, _ = gpu_solve(prob, params(p=5, tol=1e-12), b, x0=xstar)
    assert res["status"] == aar.AAR_OK and res["iterations"] == 5
    np.testing.assert_allclose(x, xstar, rtol=0, atol=1e-11 * np.abs(xstar).max())


def test_invalid_solve_leaves_x_untouched():
    import torch
    prob = inputs.dirichlet_poisson_problem(8)
    say("invalid solve")
    s = aar.Solver([prob], params())
    x = to_dev(np.full(prob.size, 7.0))
    with pytest.raises(aar.AarError) as ei:
        aar.aar_solve(s.handle, 0, x.data_ptr())
    assert ei.value.status == aar.AAR_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert (x.cpu().numpy() == 7.0).all()
    s.close()


def test_no_graph_matches_graph():
    w = inputs.workload(1)
    prob, b = w.problems[0], w.b[0]
    say("graph vs no graph")
    x1, r1, _ = gpu_solve(prob, params(tol=1e-8), b)
    x2, r2, _ = gpu_solve(prob, params(tol=1e-8, flags=aar.AAR_FLAG_NO_GRAPH), b)
    assert r1["iterations"] == r2["iterations"]
    np.testing.assert_array_equal(x1, x2)


def test_repeat_solves_are_bitwise_identical():
    w = inputs.workload(2, n=32)
    prob, b = w.problems[0], w.b[0]
    say("repeat solves")
    s = aar.Solver([prob], w.params)
    bt = to_dev(b)
    outs = []
    for _ in range(3):
        xt = to_dev(np.zeros(prob.size))
        r = s.solve(bt, xt)
        outs.append((r["iterations"], xt.cpu().numpy()))
    s.close()
    for it, xv in outs[1:]:
        assert it == outs[0][0]
        np.testing.assert_array_equal(xv, outs[0][1])


ORDER_CASES = [
    # (name, problem, (rows per thread, z depth, order bits, paired)); grids are
    # distinct so each gets its own tile-file line
    ("r3_zperiodic_order0", inputs.Problem(n=(70, 37, 45), h=(0.02, 0.03, 0.025), bc=(0, 0, 1), radius=3), (2, 8, 0, 0)),
    ("r3_zperiodic_altz", inputs.Problem(n=(70, 37, 46), h=(0.02, 0.03, 0.025), bc=(0, 0, 1), radius=3), (2, 8, 1, 0)),
    ("r3_zperiodic_zfast", inputs.Problem(n=(70, 37, 47), h=(0.02, 0.03, 0.025), bc=(0, 0, 1), radius=3), (2, 8, 2, 0)),
    ("r3_zperiodic_both", inputs.Problem(n=(70, 37, 43), h=(0.02, 0.03, 0.025), bc=(0, 0, 1), radius=3), (2, 8, 3, 0)),
    ("r6_dirichlet_altz", inputs.Problem(n=(65, 30, 41), h=(0.02, 0.03, 0.025), bc=(0, 0, 0), radius=6), (2, 8, 1, 0)),
    ("upwind_altz", cd_problem((66, 35, 29)), (2, 8, 1, 0)),
    ("upwind_both", cd_problem((66, 35, 31)), (2, 8, 3, 0)),
    # paired layout (even n0, no convection): odd and even radii, ragged y and
    # z tails, periodic x narrower than the 64-wide tile, both z directions
    ("pair_r3_ry1", inputs.Problem(n=(70, 37, 44), h=(0.02, 0.03, 0.025), bc=(0, 0, 1), radius=3), (1, 8, 0, 1)),
    ("pair_r6_ry2_dirichlet", inputs.Problem(n=(66, 30, 41), h=(0.02, 0.03, 0.025), bc=(0, 0, 0), radius=6),
     (2, 8, 1, 1)),
    ("pair_r1_dirichlet", inputs.Problem(n=(34, 20, 19), h=(0.03, 0.05, 0.05), bc=(0, 0, 0), radius=1), (1, 4, 0, 1)),
    ("pair_r4_periodic_narrow", inputs.Problem(n=(26, 25, 27), h=(1 / 26, 1 / 25, 1 / 27), bc=(1, 1, 1), radius=4,
                                               shift=0.5), (2, 8, 3, 1)),
    ("pair_r5_mixed_bc", inputs.Problem(n=(128, 19, 29), h=(0.01, 0.05, 0.04), bc=(1, 0, 1), radius=5, diffusion=0.7),
     (1, 16, 1, 1)),
    ("pair_r2_zfast", inputs.Problem(n=(96, 41, 23), h=(0.01, 0.03, 0.04), bc=(0, 1, 0), radius=2, shift=0.2),
     (2, 4, 2, 1)),
    # 512- and 1024-thread paired workgroups (the wider ones compile for FP32
    # only: the FP64 line of such a shape is rejected and FP64 is autotuned)
    ("pair8w_r6_ry1", inputs.Problem(n=(70, 37, 44), h=(0.02, 0.03, 0.025), bc=(0, 0, 1), radius=6, shift=0.3),
     (1, 8, 1, 2)),
    ("pair8w_fp32_ry2", inputs.Problem(n=(96, 45, 29), h=(0.01, 0.02, 0.03), bc=(1, 1, 1), radius=4, shift=2.0),
     (2, 8, 0, 2)),
    ("pair16w_fp32", inputs.Problem(n=(64, 70, 33), h=(0.015, 0.015, 0.03), bc=(0, 1, 0), radius=3, shift=1.0),
     (1, 12, 3, 3)),
    # an odd n0 with the paired flag falls back to the one-point layout
    ("pair_flag_odd_n0", inputs.Problem(n=(67, 29, 33), h=(1 / 67, 1 / 29, 1 / 33), bc=(1, 1, 1), radius=6),
     (1, 8, 0, 1)),
]


@pytest.mark.parametrize("name,prob,shape", ORDER_CASES, ids=[c[0] for c in ORDER_CASES])
def test_tile_order_bits_match_oracle(name, prob, shape, tmp_path, monkeypatch):
    """Every tile layout choice read from a tile file (rows per thread, z
    depth, tile numbering and z direction, paired layout) gives the oracle's
    operator and iterates, on grids whose z extent splits into an odd number
    of chunks with a short last one."""
    conv = 1 if prob.velocity is not None else 0
    ry, cz, order, pair = shape
    tile = tmp_path / "tiles.txt"
    tile.write_text(f"0 {prob.radius} {conv} {prob.n[0]} {prob.n[1]} {prob.n[2]} {ry} {cz} {order} {pair}\n"
                    f"1 {prob.radius} {conv} {prob.n[0]} {prob.n[1]} {prob.n[2]} {ry} {cz} {order} {pair}\n")
    monkeypatch.setenv("AAR_TUNE_CACHE", str(tile))
    say(f"tile shape {shape} {name} n={prob.n}")
    x = inputs.normal(17, 0, prob.size)
    s = aar.Solver([prob], params())
    y = s.apply(to_dev(x)).cpu().numpy()
    s.close()
    ref = oracle.apply(prob, x)
    scale = np.abs(oracle.diagonal(prob)).max() * np.abs(x).max()
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13 * scale)
    b = inputs.normal(5, 0, prob.size)
    for K in (5, 7, 13):
        prm = params(max_iter=K, tol=1e-30, m=7, p=6)
        xs, res, _ = gpu_solve(prob, prm, b)
        refx = oracle.aar_solve(prob, b, m=7, p=6, tol=1e-30, max_iter=K)["x"]
        np.testing.assert_allclose(xs, refx, rtol=0, atol=1e-10 * np.abs(refx).max(), err_msg=f"K={K}")
    if conv == 0 and prob.shift > 0:
        # the FP32 sweeps of the mixed path and the FP32 history of the FP64
        # path, with the same layout, reach the FP64 tolerance
        for prec in (aar.AAR_MIXED_FP32, aar.AAR_FP64_FP32HIST):
            prm = params(tol=1e-10, precision=prec)
            xm, res, _ = gpu_solve(prob, prm, b)
            assert res["status"] == aar.AAR_OK, (prec, res)
            rr = oracle.relative_residual(prob, b, xm)
            assert rr < 1e-10
            if prec == aar.AAR_MIXED_FP32:
                # the FP64 refinement residual (one-point grid whatever the
                # tile's layout) is summed over all of its partials
                assert rr == pytest.approx(res["rel_residual"], rel=1e-6), (rr, res)
