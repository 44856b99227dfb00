"""The C-ABI library loads and exports every function include/aar.h declares,
and rejects bad arguments before any device work (no GPU needed)."""
import subprocess

import pytest

from paper_1606_08740_amd import aar, inputs


def test_every_declared_symbol_is_exported():
    names = aar.header_functions()
    assert {"aar_create", "aar_solve", "aar_solve_batched", "aar_destroy", "aar_apply",
            "aar_last_error", "aar_workspace_bytes"} <= set(names)
    lib = aar.load_library()
    out = subprocess.run(["nm", "-D", "--defined-only", aar.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)


def _ws(prob, params):
    return aar.aar_workspace_bytes([aar.make_problem(prob)], aar.make_params(params))


def test_workspace_bytes_scales_with_history():
    prob = inputs.periodic_problem(32, 6)
    b7 = _ws(prob, inputs.Params(m=7, p=6))
    b10 = _ws(prob, inputs.Params(m=10, p=6))
    assert b10 - b7 >= 3 * 8 * prob.size
    mixed = _ws(prob, inputs.Params(m=7, p=6, precision=1))
    bf = _ws(prob, inputs.Params(m=7, p=6, precision=2))
    assert bf < mixed
    # FP64 iterate with a narrow history: 8 history slots of 4 or 2 bytes
    # instead of 8 (FP32 increments beside the FP32 ring; the bfloat16 ring
    # plus one FP64 copy of f_k)
    f64 = _ws(prob, inputs.Params(m=7, p=6, precision=0))
    h32 = _ws(prob, inputs.Params(m=7, p=6, precision=3))
    h16 = _ws(prob, inputs.Params(m=7, p=6, precision=4))
    assert h16 < h32 < f64
    assert f64 - h32 >= 8 * 4 * prob.size


@pytest.mark.parametrize("field,value,status", [
    ("m", 0, aar.AAR_ERR_INVALID_ARG), ("m", 33, aar.AAR_ERR_INVALID_ARG), ("p", 0, aar.AAR_ERR_INVALID_ARG),
    ("tol", 0.0, aar.AAR_ERR_INVALID_ARG), ("tol", float("nan"), aar.AAR_ERR_INVALID_ARG),
    ("max_iter", 0, aar.AAR_ERR_INVALID_ARG), ("precision", 5, aar.AAR_ERR_INVALID_ARG),
    ("precision", -1, aar.AAR_ERR_INVALID_ARG),
])
def test_bad_params_rejected(field, value, status):
    prm = inputs.Params()
    setattr(prm, field, value)
    with pytest.raises(aar.AarError) as ei:
        _ws(inputs.dirichlet_poisson_problem(8), prm)
    assert ei.value.status == status


@pytest.mark.parametrize("change,status", [
    (dict(n=(0, 4, 4)), aar.AAR_ERR_INVALID_ARG), (dict(h=(0.1, -1.0, 0.1)), aar.AAR_ERR_INVALID_ARG),
    (dict(radius=7), aar.AAR_ERR_INVALID_ARG), (dict(radius=0), aar.AAR_ERR_INVALID_ARG),
    (dict(bc=(0, 2, 0)), aar.AAR_ERR_INVALID_ARG), (dict(diffusion=0.0), aar.AAR_ERR_INVALID_ARG),
    (dict(shift=-1.0), aar.AAR_ERR_INVALID_ARG),
    (dict(bc=(1, 1, 1), radius=6, n=(12, 13, 13)), aar.AAR_ERR_UNSUPPORTED),
])
def test_bad_problem_rejected(change, status):
    prob = inputs.dirichlet_poisson_problem(8)
    for k, v in change.items():
        setattr(prob, k, v)
    with pytest.raises(aar.AarError) as ei:
        _ws(prob, inputs.Params())
    assert ei.value.status == status
    assert aar.aar_last_error() != ""
