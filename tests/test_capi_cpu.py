"""The C-ABI library loads and exports every function include/aar.h declares,
and rejects bad arguments before any device work (no GPU needed)."""
import os
import subprocess

import numpy as np
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
    (dict(radius=2, velocity=np.zeros(3 * 512)), aar.AAR_ERR_UNSUPPORTED),
    (dict(bc=(1, 0, 0), n=(1, 8, 8), velocity=np.zeros(3 * 64)), aar.AAR_ERR_UNSUPPORTED),
])
def test_bad_problem_rejected(change, status):
    prob = inputs.dirichlet_poisson_problem(8)
    for k, v in change.items():
        setattr(prob, k, v)
    # the checks run before anything is read from the velocity pointer, so a
    # non-null placeholder address stands for a device array here
    vptr = 1 if prob.velocity is not None else 0
    with pytest.raises(aar.AarError) as ei:
        aar.aar_workspace_bytes([aar.make_problem(prob, vptr)], aar.make_params(inputs.Params()))
    assert ei.value.status == status
    assert aar.aar_last_error() != ""


def test_periodic_axis_shorter_than_stencil_accepted():
    """A periodic axis with n < 2r + 1 wraps its taps (they add up)."""
    prob = inputs.Problem(n=(4, 6, 5), h=(0.25, 1 / 6, 0.2), bc=(1, 1, 1), radius=6)
    assert _ws(prob, inputs.Params()) > 0


def test_struct_layouts_match_the_header(tmp_path):
    """The C compiler's layout of the header's structs equals the binding's:
    aar_result is {status, iterations, outer_steps, rel_residual}."""
    import ctypes
    src = tmp_path / "layout.c"
    src.write_text("""#include <stdio.h>
#include <stddef.h>
#include "aar.h"
#define F(s, m) printf(#s "." #m " %zu\\n", offsetof(s, m))
int main(void) {
  F(aar_result, status); F(aar_result, iterations); F(aar_result, outer_steps); F(aar_result, rel_residual);
  printf("aar_result.size %zu\\n", sizeof(aar_result));
  F(aar_problem, n); F(aar_problem, h); F(aar_problem, bc); F(aar_problem, radius);
  F(aar_problem, diffusion); F(aar_problem, shift); F(aar_problem, velocity);
  printf("aar_problem.size %zu\\n", sizeof(aar_problem));
  F(aar_params, omega); F(aar_params, beta); F(aar_params, m); F(aar_params, p); F(aar_params, tol);
  F(aar_params, max_iter); F(aar_params, precision); F(aar_params, inner_tol); F(aar_params, max_outer);
  F(aar_params, flags);
  printf("aar_params.size %zu\\n", sizeof(aar_params));
  return 0; }
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(aar.ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, cls in [("aar_result", aar.aar_result), ("aar_problem", aar.aar_problem),
                       ("aar_params", aar.aar_params)]:
        assert int(got[f"{cname}.size"]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)
    order = [f for f, _ in aar.aar_result._fields_]
    assert order == ["status", "iterations", "outer_steps", "rel_residual"]


def test_tile_file_block_depth_field(tmp_path, monkeypatch):
    """A tile line with a temporal block depth (11th field) is accepted for
    one-point tiles; depth with a paired tile or beyond 5 is ignored (the
    library then falls back to its default shape without error)."""
    prob = inputs.dirichlet_poisson_problem(12)
    f = tmp_path / "t.txt"
    f.write_text("0 1 0 12 12 12 2 4 0 0 3\n0 1 0 13 13 13 1 4 0 1 3\n0 1 0 14 14 14 2 4 0 0 9\n")
    monkeypatch.setenv("AAR_TUNE_CACHE", str(f))
    for n in (12, 13, 14):
        assert _ws(inputs.dirichlet_poisson_problem(n), inputs.Params()) > 0


@pytest.mark.parametrize("change,status", [
    (dict(m=9), aar.AAR_ERR_UNSUPPORTED), (dict(precision=1), aar.AAR_ERR_UNSUPPORTED),
    (dict(flags=2), aar.AAR_ERR_UNSUPPORTED), (dict(p=0), aar.AAR_ERR_INVALID_ARG),
])
def test_complex_create_rejects(change, status):
    """aar_create_complex checks its arguments before any device work."""
    prm = inputs.Params()
    for k, v in change.items():
        setattr(prm, k, v)
    prob = inputs.periodic_problem(8, 3, shift=0.5)
    with pytest.raises(aar.AarError) as ei:
        aar.aar_create_complex(aar.make_problem(prob), aar.make_params(prm), -0.07)
    assert ei.value.status == status


def test_select_parameters_rejects_bad_candidates():
    prob = inputs.dirichlet_poisson_problem(8)
    for betas, ps, trial in (([], [2], 10), ([0.6], [0], 10), ([0.6], [2], 0), ([float("nan")], [2], 10)):
        with pytest.raises(aar.AarError) as ei:
            aar.aar_select_parameters(aar.make_problem(prob), aar.make_params(inputs.Params()), 1, betas, ps, trial)
        assert ei.value.status == aar.AAR_ERR_INVALID_ARG


def _csr(rowptr, col, val):
    return (np.asarray(rowptr, dtype=np.int64), np.asarray(col, dtype=np.int32), np.asarray(val, dtype=np.float64))


@pytest.mark.parametrize("matrix,pc,nblocks,change,status", [
    (_csr([0, 1, 2], [1, 0], [1.0, 1.0]), 1, 1, {}, aar.AAR_ERR_INVALID_ARG),            # no diagonal
    (_csr([0, 2, 3], [1, 0, 1], [1.0, 2.0, 3.0]), 1, 1, {}, aar.AAR_ERR_INVALID_ARG),    # unsorted row
    (_csr([0, 1, 2], [0, 2], [1.0, 1.0]), 1, 1, {}, aar.AAR_ERR_INVALID_ARG),            # column out of range
    (_csr([0, 1, 2], [0, 1], [1.0, float("nan")]), 1, 1, {}, aar.AAR_ERR_INVALID_ARG),   # non-finite value
    (_csr([0, 1, 2], [0, 1], [1.0, 1.0]), 1, 3, {}, aar.AAR_ERR_INVALID_ARG),            # nblocks > n
    (_csr([0, 1, 2], [0, 1], [1.0, 1.0]), 1, 0, {}, aar.AAR_ERR_INVALID_ARG),            # nblocks < 1
    (_csr([0, 1, 2], [0, 1], [1.0, 1.0]), 7, 1, {}, aar.AAR_ERR_INVALID_ARG),            # preconditioner
    (_csr([0, 1, 2], [0, 1], [1.0, 1.0]), 1, 1, dict(precision=1), aar.AAR_ERR_UNSUPPORTED),
    (_csr([0, 1, 2], [0, 1], [1.0, 1.0]), 0, 1, dict(flags=32), aar.AAR_ERR_UNSUPPORTED),
    (_csr(np.arange(20001), np.arange(20000), np.ones(20000)), 1, 1, {}, aar.AAR_ERR_UNSUPPORTED),  # block too big
])
def test_csr_create_rejects(matrix, pc, nblocks, change, status):
    """aar_create_csr checks the matrix and its arguments before any device work."""
    prm = inputs.Params()
    for k, v in change.items():
        setattr(prm, k, v)
    with pytest.raises(aar.AarError) as ei:
        aar.aar_create_csr(*matrix, pc, nblocks, aar.make_params(prm))
    assert ei.value.status == status


def test_tile_file_lines_pass_the_loader_rules():
    """Every line of the committed tile file passes the rules the library's
    loader applies (a line that fails them is skipped without an error, so
    its grid would silently lose its tuned shape): precision 0 (FP64),
    1 (FP32) or 2 (complex sweep), rows per thread 1, 2 or 4, a positive z
    depth, order bits 0..3, temporal depth 0..5 only for one-point tiles,
    paired shapes that are compiled (FP64: 4 waves x 1-2 rows or 8 waves x 1
    row; FP32 adds 8 waves x 2 rows and 16 waves x 1 row), and complex tiles
    one-point with at most 2 rows.  Each grid and precision appears once."""
    path = os.path.join(os.path.dirname(aar.LIB_PATH), "tuned_tiles.txt")
    seen = set()
    lines = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert lines
    for f in lines:
        assert len(f) == 11, f
        prec, radius, conv, n0, n1, n2, ry, cz, order, pair, tb = map(int, f)
        assert prec in (0, 1, 2) and 1 <= radius <= 6 and conv in (0, 1), f
        assert ry in (1, 2, 4) and cz >= 1 and 0 <= order <= 3 and 0 <= tb <= 5, f
        assert tb < 2 or pair == 0, f
        f64 = prec != 1
        ok = {0: True, 1: ry in (1, 2), 2: ry == 1 or (not f64 and ry == 2), 3: not f64 and ry == 1}.get(pair, False)
        assert ok, f
        if prec == 2:
            assert pair == 0 and tb == 0 and ry <= 2 and conv == 0, f
        key = (prec, radius, conv, n0, n1, n2)
        assert key not in seen, f
        seen.add(key)
