"""The seeded input generators: published SplitMix64 values, determinism and
the stated shapes and distributions of each workload."""
import numpy as np

from paper_1606_08740_amd import inputs


def test_splitmix64_published_sequence():
    # SplitMix64 with state 0: first outputs as published with the generator
    # (Steele, Lea, Flood 2014; the reference C implementation by Vigna).
    z = inputs.splitmix64(0, 3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_streams_deterministic_and_distinct():
    a = inputs.normal(3, 0, 1000)
    np.testing.assert_array_equal(a, inputs.normal(3, 0, 1000))
    assert not np.array_equal(a, inputs.normal(3, 1, 1000))
    u = inputs.uniform(9, 2, 200000)
    assert 0.0 <= u.min() and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01
    g = inputs.normal(9, 2, 200000)
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1.0) < 0.01


def test_workload_shapes():
    w = inputs.workload(1)
    assert w.problems[0].n == (32, 32, 32) and w.params.tol == 1e-8 and (w.params.m, w.params.p) == (7, 6)
    assert abs(w.problems[0].h[0] - 1 / 33) < 1e-17
    b = inputs.gaussian_charges(24, 2)
    assert abs(b.mean()) < 1e-15 * np.abs(b).max() and b.shape == (24 ** 3,)
    v = inputs.convection_field(20, 4)
    h = 1 / 21
    assert abs(np.abs(v).max() * h / 2 - 0.5) < 1e-12
    wb = inputs.batched_helmholtz(count=40)
    ns = [p.n[0] for p in wb.problems]
    assert min(ns) >= 16 and max(ns) <= 96
    assert all(0 < p.shift < 10 for p in wb.problems)
    assert all(p.radius == 4 and p.bc == (1, 1, 1) for p in wb.problems)


def test_tile_tuner_keeps_lines_it_did_not_tune():
    """Re-tuning some grids rewrites their lines and keeps every other line
    of the tile file (batch lines, complex lines, other grids) in order."""
    from paper_1606_08740_amd import tune_tiles
    old = ("# header\n0 6 0 192 192 192 1 28 0 2 0\n1 6 0 192 192 192 1 16 1 2 0\n"
           "0 4 0 0 0 0 2 32 0 0 0\n2 3 0 72 72 72 1 4 2 0 0\n")
    new = ["1 6 0 192 192 192 1 16 0 2 0\n", "0 1 0 32 32 32 1 2 1 1 0\n"]
    out = tune_tiles.merge_lines(old, new).splitlines()
    assert out[0].startswith("#")
    assert out[1:] == ["0 6 0 192 192 192 1 28 0 2 0", "0 4 0 0 0 0 2 32 0 0 0", "2 3 0 72 72 72 1 4 2 0 0",
                       "1 6 0 192 192 192 1 16 0 2 0", "0 1 0 32 32 32 1 2 1 1 0"]
