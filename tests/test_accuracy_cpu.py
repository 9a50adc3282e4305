"""The accuracy metrics (paper_1003_3896_amd.accuracy) on hand-made arrays whose errors are known
exactly, and the bench's row sampler."""
import math

import numpy as np

from paper_1003_3896_amd import accuracy


def test_metrics_on_known_errors():
    # two clusters: rows 0-1 (|r| = 3, 4) and rows 2-3 (|r| = 1, 1)
    ref = np.array([[3.0, 0, 0], [0, 4.0, 0], [1.0, 0, 0], [0, 0, 1.0]])
    a = ref.copy()
    a[1, 1] += 0.4   # |da| = 0.4 on |r| = 4
    a[2, 2] -= 0.1   # |da| = 0.1 on |r| = 1
    scale = np.array([6.0, 8.0, 2.0, 1.0])
    st = accuracy.accel_error(a, ref, offsets=[0, 2, 4], scale=scale)
    arms0 = math.sqrt((9 + 16) / 2)
    assert st["rows"] == 4
    assert abs(st["max_over_arms"] - max(0.4 / arms0, 0.1 / 1.0)) < 1e-15
    assert abs(st["l2"] - math.sqrt((0.16 + 0.01) / (9 + 16 + 1 + 1))) < 1e-15
    assert abs(st["rel_max"] - 0.1) < 1e-15
    assert abs(st["rel_median"] - 0.05) < 1e-15  # per-particle errors 0, 0.1, 0.1, 0
    assert abs(st["s_max"] - 0.05) < 1e-15 and st["s_median"] == 0.025
    # a_rms supplied per cluster (from a full reference) instead of the sampled rows
    st2 = accuracy.accel_error(a, ref, offsets=[0, 2, 4], arms=[10.0, 1.0])
    assert abs(st2["max_over_arms"] - 0.1) < 1e-15
    # rows of a larger batch: cluster membership follows the given row indices
    st3 = accuracy.accel_error(a, ref, offsets=[0, 100, 200], rows=[5, 6, 150, 151])
    assert abs(st3["max_over_arms"] - st["max_over_arms"]) < 1e-15


def test_zero_reference_rows():
    ref = np.zeros((3, 3))
    ref[0, 0] = 1.0
    a = ref.copy()
    st = accuracy.accel_error(a, ref, scale=np.array([1.0, 0.0, 0.0]))
    assert st["max_over_arms"] == 0.0 and st["s_max"] == 0.0 and st["rel_max"] == 0.0
    a[1, 0] = 1e-3  # an error where the scale vanishes is infinite in the S_i metric
    assert accuracy.accel_error(a, ref, scale=np.array([1.0, 0.0, 0.0]))["s_max"] == math.inf
    assert np.isinf(accuracy.s_errors(a, ref, np.array([1.0, 0.0, 0.0]))[1])


def test_gates():
    ok = {"s_max": 5e-7, "s_median": 1e-8}
    assert accuracy.gate(ok, "fp32dl") and accuracy.gate(ok, "fp32ds") and not accuracy.gate(ok, "fp64")
    assert not accuracy.gate({"s_max": 2e-6, "s_median": 1e-8}, "fp32ds")
    assert accuracy.gate({"s_max": 4e-5, "s_median": 2e-8}, "fp32c")


def test_bench_row_sampler():
    import bench
    idx = bench.sample_rows(262144, 2048)
    assert len(idx) == 3 * (2048 // 3) and idx[0] == 0 and idx[-1] == 262143
    assert np.all(np.diff(idx) > 0)
    assert np.array_equal(bench.sample_rows(100, 2048), np.arange(100))
