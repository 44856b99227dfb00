"""The allocation-free entry point (aar_solve_noalloc) against aar_solve.

aar_solve_noalloc runs the FP64 solve of aar_solve with its workspace in a
fixed device array instead of device allocations, and the default tile
shapes.  Through the C ABI, each call here is compared with aar_solve on a
handle created with AAR_FLAG_NO_AUTOTUNE (the same kernels and tiles): the
answers agree bit for bit, and so do the status, iteration count and
residual.  The calls run back to back with the later systems smaller, so the
array holds the previous call's data when a call starts.
"""
import numpy as np
import pytest

from paper_1606_08740_amd import aar, inputs
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def handle_solve(prob, prm, b):
    import torch
    s = aar.Solver([prob], prm)
    bt = to_dev(b)
    xt = torch.zeros_like(bt)
    res = s.solve(bt, xt)
    torch.cuda.synchronize()
    s.close()
    return xt.cpu().numpy(), res


def noalloc_solve(prob, prm, b, vel=None):
    import torch
    bt = to_dev(b)
    xt = torch.zeros_like(bt)
    vt = to_dev(vel) if vel is not None else None
    stream = torch.cuda.current_stream().cuda_stream
    r = aar.aar_solve_noalloc(aar.make_problem(prob, vt.data_ptr() if vt is not None else 0),
                              aar.make_params(prm), bt.data_ptr(), xt.data_ptr(), stream)
    torch.cuda.synchronize()
    return xt.cpu().numpy(), aar.result_dict(r)


CASES = [
    ("periodic_r6_44_shift", lambda: (inputs.Problem(n=(44, 44, 44), h=(1 / 44,) * 3, bc=(1, 1, 1), radius=6,
                                                     shift=0.3), 1e-10)),
    ("dirichlet_7pt_32", lambda: (inputs.dirichlet_poisson_problem(32), 1e-8)),
    ("upwind_20", lambda: (inputs.workload(4, n=20, precision=0).problems[0], 1e-10)),
    ("periodic_r4_odd_18", lambda: (inputs.Problem(n=(19, 18, 17), h=(1 / 19, 1 / 18, 1 / 17), bc=(1, 1, 1),
                                                   radius=4, shift=2.0), 1e-10)),
]


def test_noalloc_matches_handle_solve_on_shrinking_calls():
    for name, make in CASES:
        prob, tol = make()
        b = inputs.normal(31, 0, prob.size)
        m, p = (10, 4) if prob.velocity is not None else (7, 6)
        prm = inputs.Params(m=m, p=p, tol=tol, flags=aar.AAR_FLAG_NO_AUTOTUNE)
        say(f"no-alloc {name} n={prob.n}")
        x1, r1 = noalloc_solve(prob, prm, b, prob.velocity)
        x0, r0 = handle_solve(prob, prm, b)
        assert r0["status"] == aar.AAR_OK, r0
        assert r1 == r0, (r1, r0)
        np.testing.assert_array_equal(x1, x0)


def test_noalloc_rejects_oversize_and_other_modes():
    import torch
    big = inputs.dirichlet_poisson_problem(80)
    bt = torch.zeros(big.size, dtype=torch.float64, device="cuda:0")
    xt = torch.full_like(bt, 3.0)
    with pytest.raises(aar.AarError) as ei:
        aar.aar_solve_noalloc(aar.make_problem(big), aar.make_params(inputs.Params()), bt.data_ptr(), xt.data_ptr())
    assert ei.value.status == aar.AAR_ERR_UNSUPPORTED
    small = inputs.dirichlet_poisson_problem(16)
    for prm in (inputs.Params(precision=1), inputs.Params(flags=aar.AAR_FLAG_RECORD_RESIDUALS)):
        with pytest.raises(aar.AarError) as ei:
            aar.aar_solve_noalloc(aar.make_problem(small), aar.make_params(prm), bt.data_ptr(), xt.data_ptr())
        assert ei.value.status == aar.AAR_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert (xt.cpu().numpy() == 3.0).all()
