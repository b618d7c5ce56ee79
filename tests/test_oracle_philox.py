"""Pins of the oracle's counter-based Gaussian source: the published
Philox4x32-10 known-answer vectors (golden fixture) and the moments of the
Box-Muller samples."""
import json
import os

import numpy as np

from oracle.philox import philox4x32_10, gaussian_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox_kat.json")


def test_philox_known_answer_vectors():
    for v in json.load(open(GOLDEN))["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = [int(x) for x in philox4x32_10(ctr, key)]
        assert out == [int(x, 16) for x in v["out"]]


def test_gaussian_matrix_moments_and_determinism():
    g = gaussian_matrix(400, seed=123, tag=0)
    assert g.shape == (400, 400) and g.flags["F_CONTIGUOUS"]
    x = g.ravel()
    assert abs(x.mean()) < 5.0 / 400
    assert abs(x.var() - 1.0) < 0.02
    assert abs(np.mean(x ** 4) - 3.0) < 0.1
    assert np.array_equal(g, gaussian_matrix(400, seed=123, tag=0))
    assert not np.array_equal(g, gaussian_matrix(400, seed=123, tag=1))
    assert not np.array_equal(g, gaussian_matrix(400, seed=124, tag=0))
    # element (i, j) does not depend on n: keyed by the column-major index
    small = gaussian_matrix(3, seed=123, tag=0)
    assert small[0, 0] == g[0, 0] and small[1, 0] == g[1, 0]
