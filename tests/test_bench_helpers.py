"""Host-side helpers of bench.py: the tile lookup that decides whether the
profiled sweep traffic applies, and the error against the oracle's stored
solution samples (tests/golden/oracle_full_size.json, written by the oracle
only)."""
import json
import os

import numpy as np
import pytest

import bench

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_full_size.json")


def test_fp64_tile_reads_the_tile_file(tmp_path, monkeypatch):
    f = tmp_path / "tiles.txt"
    f.write_text("# comment\n1 6 0 192 192 192 2 8 1 1\n0 6 0 192 192 192 1 20 3 2\n0 4 0 192 192 192 4 4\n")
    monkeypatch.setenv("AAR_TUNE_CACHE", str(f))
    assert bench.fp64_tile(192) == {"rows_per_thread": 1, "z_depth": 20, "order": 3, "pair": 2}
    assert bench.fp64_tile(192, radius=4) == {"rows_per_thread": 4, "z_depth": 4, "order": 0, "pair": 0}
    assert bench.fp64_tile(256) is None


def test_sweep_traffic_only_for_the_profiled_tile(tmp_path, monkeypatch):
    monkeypatch.delenv("AAR_TUNE_CACHE", raising=False)
    t = bench.sweep_traffic(192)
    if t is not None:   # the committed profile matches the committed tile and sources
        # between the recursion sweeps' algorithmic bytes (17.6 B per point)
        # and twice the direct sweep's (32 B per point)
        assert 17.6 * 192 ** 3 < t < 2 * 32 * 192 ** 3
    assert bench.sweep_traffic(128) is None
    f = tmp_path / "tiles.txt"
    f.write_text("0 6 0 192 192 192 4 2 0 0\n")   # a shape no profile was taken with
    monkeypatch.setenv("AAR_TUNE_CACHE", str(f))
    assert bench.sweep_traffic(192) is None


def test_oracle_sample_error():
    g = json.load(open(GOLDEN))["periodic_poisson_r6_192"]
    n = 192 ** 3
    rms = g["x_norm"] / np.sqrt(n)
    x = np.zeros(n)
    idx = np.asarray(g["sample_index"])
    x[idx] = g["sample_x"]
    x += 0.25          # a constant offset is invisible in a mean-free comparison
    assert bench.oracle_sample_error(x, 192) < 1e-5
    x[idx[3]] += 1e-3 * rms
    assert bench.oracle_sample_error(x, 192) == pytest.approx(1e-3, rel=1e-2)
    assert bench.oracle_sample_error(x, 100) is None


def test_byte_models():
    """Per-point byte counts of the design's passes (m = 7, p = 6, FP64):
    sweeps 24 + 4 x 16, residual + fused Gram 64, update 96 = 248 B per cycle;
    with the separate Gram pass 16 + 64 for the residual and the products."""
    assert bench.sweep_bytes_per_point(7, 6) == pytest.approx(17.6)
    assert bench.sweep_bytes_per_point(3, 6) == 32.0        # ring shorter than a cycle: direct sweeps
    assert bench.cycle_bytes(bench.FP64, 7, 6, fused_gram=True) == 248
    assert bench.cycle_bytes(bench.FP64, 7, 6) == 264
    # FP64 iterate with an FP32 ring: first sweep 8 + 8 + 4, then 4 x 8 over
    # the ring and the residual 8, Gram 8 x 4, update 8 + 32 + 4 + 8 + 4
    assert bench.cycle_bytes(bench.FP64_FP32HIST, 7, 6) == 20 + 4 * 8 + 8 + 32 + 56
    assert bench.cycle_bytes(bench.MIXED, 7, 6) == 12 + 4 * 8 + 8 + 32 + 4 + 32 + 4 + 4 + 4
    assert bench.cycle_bytes(bench.FP64_BF16HIST, 7, 6) is None


def test_complex_byte_model():
    # 5 sweeps x 64 + residual 48 + Gram 8 x 16 + update 16 + 128 + 16 + 32
    assert bench.complex_cycle_bytes(7, 6) == 5 * 64 + 48 + 128 + 192


def test_csr_sweep_bytes():
    """A's values, columns and row pointers once, x, b, new x and f, plus the
    ILU(0) factors with their columns."""
    import bench
    assert bench.csr_sweep_bytes(10, 50) == 12 * 50 + 8 * 11 + 32 * 10
    assert bench.csr_sweep_bytes(10, 50, 40) == bench.csr_sweep_bytes(10, 50) + 12 * 40


@pytest.mark.parametrize("key", ["ofdft_helmholtz_72", "ofdft_helmholtz_144", "reservoir_128_jacobi",
                                 "reservoir_128_block_ilu0_1024", "periodic_poisson_r6_256"])
def test_stored_oracle_solutions_are_converged(key):
    """Every stored full-size oracle solution the benchmark compares against
    converged to its tolerance and keeps 64 seeded sample points."""
    g = json.load(open(GOLDEN))[key]
    assert g["status"] == 0 and g["relres"] < g["tol"]
    assert len(g["sample_index"]) == 64
    assert g["iterations"] > 0
