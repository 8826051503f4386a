"""Pins for the similarity-threshold queries of the oracle (the method needs
only a yes/no similarity query per sampled pair, Section 1): an edge when the
binary64 dot product, or the binary64 cosine, of the pair is at least tau.

Each pin comes from outside the oracle's own formula: exact rational
arithmetic step by step, integer data whose sums are exact in any order
(checked against a brute-force DBSCAN), exact ties, the scale invariance of
the cosine, and the polarisation identity <a,b> = (|a|^2 + |b|^2 - |a-b|^2)/2,
which ties the dot-product query to the distance query on rows of equal norm.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from bruteforce import dbscan_adjacency


def _f32(X):
    return np.asarray(X, np.float32)


def _exact_dot(a, b):
    """Sequential binary64 dot product, each rounding done by exact rationals."""
    acc = 0.0
    for x, y in zip(a, b):
        p = float(Fraction(float(x)) * Fraction(float(y)))
        acc = float(Fraction(acc) + Fraction(p))
    return acc


def test_dot_is_binary64_sequential(orc):
    rng = np.random.default_rng(11)
    for _ in range(300):
        d = int(rng.integers(1, 40))
        X = (rng.normal(size=(2, d)) * 10.0 ** rng.integers(-15, 15)).astype(np.float32)
        assert orc.dot(X, 0, 1) == _exact_dot(X[0], X[1])


def test_cosine_rounding(orc):
    """cosine = fl(ip / fl(fl(sqrt(Ni)) * fl(sqrt(Nj)))): quotient and product
    rounded once each by exact rationals; math.sqrt is correctly rounded."""
    rng = np.random.default_rng(12)
    for _ in range(300):
        d = int(rng.integers(1, 30))
        X = (rng.normal(size=(2, d)) * 10.0 ** rng.integers(-8, 8)).astype(np.float32)
        ip = _exact_dot(X[0], X[1])
        ni = math.sqrt(_exact_dot(X[0], X[0]))
        nj = math.sqrt(_exact_dot(X[1], X[1]))
        den = float(Fraction(ni) * Fraction(nj))
        assert orc.cosine(X, 0, 1) == float(Fraction(ip) / Fraction(den))


def test_dot_tie_and_next_value(orc):
    X = _f32([[3, 4, 0], [4, 3, 5]])  # dot = 24 exactly
    r = orc.dbscan_similarity(X, orc.DOT, 24.0, 1, exhaustive=True)
    assert r.deg.tolist() == [1, 1] and r.labels.tolist() == [0, 0]
    r = orc.dbscan_similarity(X, orc.DOT, math.nextafter(24.0, 25.0), 1, exhaustive=True)
    assert r.deg.tolist() == [0, 0] and r.labels.tolist() == [-1, -1]


def test_cosine_tie_and_next_value(orc):
    # cos((3,4),(4,3)) = 24/25: both the method and the literal 0.96 are the
    # correctly rounded value of 24/25
    X = _f32([[3, 4], [4, 3]])
    assert orc.cosine(X, 0, 1) == 0.96
    assert orc.dbscan_similarity(X, orc.COSINE, 0.96, 1, exhaustive=True).deg.tolist() == [1, 1]
    r = orc.dbscan_similarity(X, orc.COSINE, math.nextafter(0.96, 1.0), 1, exhaustive=True)
    assert r.deg.tolist() == [0, 0]


def test_zero_rows(orc):
    """A zero row has no cosine (0/0) and so no edge at any tau; its dot
    product with anything is 0, an edge exactly when tau <= 0."""
    X = _f32([[0, 0, 0], [1, 2, 3], [0, 0, 0], [-1, 0.5, 2]])
    r = orc.dbscan_similarity(X, orc.COSINE, -1e300, 1, exhaustive=True)
    assert r.deg.tolist() == [0, 1, 0, 1]
    assert math.isnan(orc.cosine(X, 0, 1)) and math.isnan(orc.cosine(X, 0, 2))
    r = orc.dbscan_similarity(X, orc.DOT, 0.0, 1, exhaustive=True)
    assert r.deg[0] == 3 and r.deg[2] == 3
    r = orc.dbscan_similarity(X, orc.DOT, math.nextafter(0.0, 1.0), 1, exhaustive=True)
    assert r.deg[0] == 0 and r.deg[2] == 0


def test_nan_rows_have_no_edges(orc):
    X = _f32([[1, 1], [np.nan, 1], [2, 2], [np.inf, 0]])
    for kind in (orc.DOT, orc.COSINE):
        r = orc.dbscan_similarity(X, kind, -1e300, 1, exhaustive=True)
        assert r.deg[1] == 0 and (kind == orc.DOT or r.deg[3] == 0)
        assert r.deg[0] >= 1 and r.deg[2] >= 1


def test_exhaustive_dot_matches_bruteforce_on_integers(orc):
    """Small integers: every product and partial sum is exact in binary64,
    so the integer Gram matrix decides each pair whatever the order."""
    rng = np.random.default_rng(13)
    for n, d, tau, mp in [(60, 5, 20.0, 3), (80, 3, 0.0, 4), (50, 8, -10.0, 10), (70, 2, 30.0, 2)]:
        Xi = rng.integers(-8, 9, size=(n, d))
        G = Xi @ Xi.T
        want_labels, want_deg, _ = dbscan_adjacency(G >= tau, mp)
        r = orc.dbscan_similarity(_f32(Xi), orc.DOT, tau, mp, exhaustive=True)
        assert np.array_equal(r.deg, want_deg) and np.array_equal(r.labels, want_labels)


def _integer_norm_rows():
    """Integer 3-vectors of integer length (Pythagorean quadruples), with
    sign changes and coordinate permutations."""
    base = [(1, 2, 2), (2, 3, 6), (1, 4, 8), (4, 4, 7), (2, 6, 9), (3, 4, 12), (0, 3, 4),
            (2, 10, 11), (6, 6, 7), (0, 5, 12)]
    rows = set()
    for v in base:
        for p in itertools.permutations(v):
            for s in itertools.product((1, -1), repeat=3):
                rows.add(tuple(a * b for a, b in zip(p, s)))
    return np.array(sorted(rows), np.int64)


def test_exhaustive_cosine_matches_exact_rationals(orc):
    """With integer rows of integer norm, ip and the norm product are exact
    integers, so the method's cosine is the correctly rounded rational
    ip / (|a||b|), which Python's Fraction-to-float conversion gives
    independently. tau = 0.8 (the ratio 4/5 rounds to it) and a tau taken
    from one pair's ratio are ties, where only the rounded quotient decides."""
    R = _integer_norm_rows()
    rng = np.random.default_rng(14)
    R = R[rng.choice(len(R), 90, replace=False)]
    norms = np.round(np.sqrt((R * R).sum(1))).astype(np.int64)
    assert np.array_equal(norms * norms, (R * R).sum(1))
    G = R @ R.T
    q = np.array([[float(Fraction(int(G[i, j]), int(norms[i] * norms[j])))
                   for j in range(len(R))] for i in range(len(R))])
    tie = float(q[3, 7])  # a pair sits exactly on this tau
    for tau, mp in [(tie, 3), (0.8, 2), (-0.2, 6), (0.93, 1)]:
        want_labels, want_deg, _ = dbscan_adjacency(q >= tau, mp)
        r = orc.dbscan_similarity(_f32(R), orc.COSINE, tau, mp, exhaustive=True)
        assert np.array_equal(r.deg, want_deg) and np.array_equal(r.labels, want_labels)
    assert (q == 0.8).any()  # 4/5 rounds to the literal 0.8: a tie as well


def test_cosine_is_scale_invariant(orc):
    """Scaling a row by a power of two scales its dot products and its norm
    exactly, so every cosine, and so the whole sampled result, is unchanged."""
    rng = np.random.default_rng(15)
    X = rng.normal(size=(400, 6)).astype(np.float32)
    k = rng.integers(-20, 21, size=(400, 1))
    Xs = (X * np.ldexp(np.float32(1.0), k)).astype(np.float32)
    for tau in (0.3, 0.9, -0.5):
        a = orc.dbscan_similarity(X, orc.COSINE, tau, 4, seed=3, m=25)
        b = orc.dbscan_similarity(Xs, orc.COSINE, tau, 4, seed=3, m=25)
        assert np.array_equal(a.deg, b.deg) and np.array_equal(a.labels, b.labels)
        assert a.accepted > 0


def test_dot_equals_distance_on_equal_norms(orc):
    """Polarisation: on rows of equal squared norm N, <a,b> >= tau exactly
    when |a-b|^2 <= 2N - 2tau. Signed permutations of (0,3,4) all have N = 25
    and integer coordinates, so both sides are exact; tau = 17 is eps = 4 and
    tau = 12.5 is eps = 5."""
    R = np.array(sorted({tuple(a * b for a, b in zip(p, s))
                         for p in itertools.permutations((0, 3, 4))
                         for s in itertools.product((1, -1), repeat=3)}), np.float32)
    rng = np.random.default_rng(16)
    X = R[rng.integers(0, len(R), size=500)]
    for tau, eps in [(17.0, 4.0), (12.5, 5.0), (-25.0, 10.0)]:
        for seed, m, mp in [(1, 30, 5), (7, 9, 3)]:
            a = orc.dbscan_similarity(X, orc.DOT, tau, mp, seed=seed, m=m)
            b = orc.dbscan(X, eps, mp, seed, m=m)
            assert np.array_equal(a.deg, b.deg) and np.array_equal(a.labels, b.labels)
            assert a.accepted == b.accepted and a.self_pairs == b.self_pairs


def test_dot_with_tau_below_everything_accepts_every_slot(orc):
    """tau far below any dot product: every non-self slot is an edge, the
    same graph as the distance query with a huge eps."""
    rng = np.random.default_rng(17)
    X = rng.normal(size=(300, 4)).astype(np.float32)
    a = orc.dbscan_similarity(X, orc.DOT, -1e30, 3, seed=9, m=11)
    b = orc.dbscan(X, 1e30, 3, 9, m=11)
    assert a.accepted == 300 * 11 - a.self_pairs
    assert np.array_equal(a.deg, b.deg) and np.array_equal(a.labels, b.labels)


def test_out_degree_mode_similarity(orc):
    """Out-degrees plus in-degrees are the symmetrised degrees; components
    use the same graph."""
    rng = np.random.default_rng(18)
    X = rng.normal(size=(500, 5)).astype(np.float32)
    for kind, tau in [(orc.DOT, 1.0), (orc.COSINE, 0.6)]:
        sym = orc.dbscan_similarity(X, kind, tau, 1, seed=4, m=40)
        out = orc.dbscan_similarity(X, kind, tau, 1, seed=4, m=40, out_degree=True)
        js = np.array([[orc.partner(4, 500, i, t) for t in range(40)] for i in range(500)])
        inn = np.zeros(500, np.int64)
        for i in range(500):
            for j in js[i]:
                if j != i and (orc.dot(X, i, j) >= tau if kind == orc.DOT
                               else orc.cosine(X, i, j) >= tau):
                    inn[j] += 1
        assert np.array_equal(out.deg.astype(np.int64) + inn, sym.deg.astype(np.int64))


def test_invalid_similarity_arguments(orc):
    X = np.zeros((3, 2), np.float32)
    for kind, tau in [(0, 1.0), (3, 1.0), (orc.DOT, float("nan")), (orc.COSINE, float("inf")),
                      (orc.DOT, float("-inf"))]:
        with pytest.raises(orc.OracleError):
            orc.dbscan_similarity(X, kind, tau, 1, m=1)
