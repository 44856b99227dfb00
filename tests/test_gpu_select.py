"""beta / p selection by timed trial solves (aar_select_parameters): the
chosen pair is one of the candidates and carries the best score; every trial
is a plain AAR solve (its iterates are the ones the parity tests pin); the
chosen parameters solve the system to tolerance, with the residual checked by
the oracle's operator."""
import numpy as np
import pytest

import oracle
from paper_1606_08740_amd import aar, inputs
from tests.gpu_util import gpu_solve, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,prob", [
    ("dirichlet_7pt_24", inputs.dirichlet_poisson_problem(24)),
    ("helmholtz_r4_20", inputs.periodic_problem(20, 4, shift=2.0)),
], ids=["dirichlet_7pt_24", "helmholtz_r4_20"])
def test_selection_returns_best_candidate_and_solves(name, prob):
    b = inputs.normal(41, 0, prob.size)
    bt = to_dev(b)
    prm = inputs.Params(tol=1e-10, flags=aar.AAR_FLAG_NO_AUTOTUNE)
    betas, ps = [0.3, 0.6, 1.0], [2, 6]
    say(f"select beta/p {name}")
    beta, p, scores = aar.aar_select_parameters(aar.make_problem(prob), aar.make_params(prm), bt.data_ptr(),
                                                 betas, ps, 60)
    assert scores.shape == (2, 3) and (scores >= 0).all() and scores.max() > 0
    assert beta in betas and p in ps
    j, i = ps.index(p), betas.index(beta)
    assert scores[j, i] == scores.max()
    prm.beta, prm.p = beta, p
    x, res, _ = gpu_solve(prob, prm, b)
    assert res["status"] == aar.AAR_OK
    assert oracle.relative_residual(prob, b, x) < prm.tol
