"""Mesh / phase pins: inclusion element counts of the workloads' microstructures."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("n,count", [(8, 12), (16, 52), (32, 208)])
def test_circle_counts(n, count):
    ph = oracle.phase_by_centroid(2, n, 0.25)
    assert int(ph.sum()) == count
    # brute-force check of the rule |centroid - c| < r
    c = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(c, c, indexing="xy")
    ref = ((X - 0.5) ** 2 + (Y - 0.5) ** 2 < 0.25 ** 2).astype(np.uint8).reshape(-1)
    assert np.array_equal(ph, ref)


def test_sphere_is_symmetric_and_x_fastest():
    n = 8
    ph = oracle.phase_by_centroid(3, n, 0.3).reshape(n, n, n)  # [k][j][i]
    assert np.array_equal(ph, ph.transpose(0, 2, 1))
    assert np.array_equal(ph, ph[::-1])
    # off-centre inclusion: only x-index shifts
    ph2 = oracle.phase_by_centroid(3, n, 0.2, center=[0.25, 0.5, 0.5]).reshape(n, n, n)
    assert ph2[4, 4, 1] == 1 and ph2[4, 4, 6] == 0
