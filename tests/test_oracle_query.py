"""Pins for the similarity query of Algorithm 1 (|x - x'| <= eps, squared,
binary64) and for the degree accumulation of the sampling step."""
import math
from fractions import Fraction

import numpy as np
import pytest


def _run(orc, X, eps, min_pts=1, m=None, exhaustive=True, seed=0):
    return orc.dbscan(np.asarray(X, np.float32), eps, min_pts, seed, m=m, exhaustive=exhaustive)


def test_exact_tie_is_accepted(orc):
    # |(0,0)-(3,4)| = 5 exactly: inclusive comparison accepts it
    r = _run(orc, [[0, 0], [3, 4]], 5.0)
    assert r.deg.tolist() == [1, 1] and r.accepted == 1


def test_next_ulp_is_rejected(orc):
    y = np.nextafter(np.float32(4.0), np.float32(np.inf))
    r = _run(orc, [[0, 0], [3, y]], 5.0)
    assert r.deg.tolist() == [0, 0]


def test_eps_just_below_tie_rejected(orc):
    r = _run(orc, [[0, 0], [3, 4]], math.nextafter(5.0, 0.0))
    assert r.deg.tolist() == [0, 0]


def test_duplicates_accepted_at_eps_zero(orc):
    r = _run(orc, [[1.5, -2.0], [1.5, -2.0], [1.5, -2.000001]], 0.0)
    assert r.deg.tolist() == [1, 1, 0]


def test_nan_and_inf_never_accepted(orc):
    X = [[0.0, 0.0], [np.nan, 0.0], [np.inf, 0.0], [0.0, 0.0]]
    r = _run(orc, X, 1e30)
    assert r.deg.tolist() == [1, 0, 0, 1]


def test_self_samples_add_nothing(orc):
    # n=1: every sample is the point itself
    r = orc.dbscan(np.zeros((1, 3), np.float32), 1e30, 0, seed=5, m=37)
    assert r.deg.tolist() == [0] and r.self_pairs == 37 and r.slots == 37
    assert r.labels.tolist() == [0]


def test_distance_is_binary64_sequential(orc):
    """D is the correctly rounded sequential binary64 sum of squared binary64
    differences; checked against exact rational arithmetic step by step."""
    rng = np.random.default_rng(3)
    for _ in range(300):
        d = int(rng.integers(1, 40))
        X = (rng.normal(size=(2, d)) * 10.0 ** rng.integers(-20, 20)).astype(np.float32)
        acc = 0.0
        for k in range(d):
            delta = float(Fraction(float(X[0, k])) - Fraction(float(X[1, k])))
            sq = float(Fraction(delta) * Fraction(delta))
            acc = float(Fraction(acc) + Fraction(sq))
        assert orc.sqdist(X, 0, 1) == acc


def test_binary64_decides_where_binary32_would_not(orc):
    # 1 + 2^-23 and 1 differ by one float ulp; their squared distance 2^-46 is
    # exact in binary64. eps^2 just below it must reject, at it must accept.
    X = np.array([[1.0], [1.0 + 2.0 ** -23]], np.float32)
    D = 2.0 ** -46
    assert orc.sqdist(X, 0, 1) == D
    assert _run(orc, X, math.sqrt(D)).deg.tolist() == [1, 1]
    assert _run(orc, X, math.nextafter(math.sqrt(D), 0)).deg.tolist() == [0, 0]


def test_degrees_are_symmetrised_with_huge_eps(orc):
    """With every non-self sample accepted, deg[i] = (m - self_i) + in_i,
    where in_i counts samples of other points that landed on i."""
    rng = np.random.default_rng(5)
    for n, m, seed in [(1, 4, 0), (2, 9, 1), (17, 13, 2), (300, 7, 3), (64, 64, 2**63 + 5)]:
        X = rng.normal(size=(n, 3)).astype(np.float32)
        r = orc.dbscan(X, 1e30, 1, seed, m=m)
        js = np.array([[orc.partner(seed, n, i, t) for t in range(m)] for i in range(n)],
                      np.int64).reshape(n, m)
        self_i = (js == np.arange(n)[:, None]).sum(1)
        inn = np.zeros(n, np.int64)
        for i in range(n):
            for j in js[i]:
                if j != i:
                    inn[j] += 1
        assert np.array_equal(r.deg.astype(np.int64), (m - self_i) + inn)
        assert r.self_pairs == int(self_i.sum()) and r.slots == n * m
        assert int(r.deg.sum()) == 2 * r.accepted


def test_invalid_arguments(orc):
    X = np.zeros((3, 2), np.float32)
    with pytest.raises(orc.OracleError):
        orc.dbscan(X, -1.0, 1, m=1)
    with pytest.raises(orc.OracleError):
        orc.dbscan(X, float("inf"), 1, m=1)
    with pytest.raises(orc.OracleError):
        orc.dbscan(X, float("nan"), 1, m=1)
    with pytest.raises(orc.OracleError):
        orc.dbscan(X, 1.0, 1, m=-1)
