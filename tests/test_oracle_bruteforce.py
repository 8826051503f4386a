"""Pins the oracle's whole pipeline at full sampling against textbook DBSCAN:
(a) an independent numpy/BFS brute force on integer grids, where every squared
distance is exact in binary64 so the two agree bit for bit; (b) scikit-learn's
DBSCAN on tie-free random inputs (cores, core partition and noise are unique;
sklearn's border choice follows its expansion order, so borders are checked
for validity only)."""
import numpy as np
import pytest

from paper_2006_06743_amd.workloads import random_instance
from tests.bruteforce import dbscan_bruteforce, pairwise_sq


@pytest.mark.parametrize("d", [1, 2, 3, 7])
def test_exhaustive_equals_bruteforce_on_grids(orc, d):
    rng = np.random.default_rng(100 + d)
    for trial in range(6):
        n = int(rng.choice([0, 1, 2, 5, 60, 400, 1200]))
        X = random_instance(rng, n, d, "grid")
        eps = float(rng.choice([0.0, 1.0, 2.0, np.sqrt(5.0), 3.0, 4.5]))
        for min_pts in [-1, 0, 1, 2, 5, 10]:
            want_l, want_d, _ = dbscan_bruteforce(X, eps, min_pts)
            r = orc.dbscan(X, eps, min_pts, exhaustive=True)
            assert np.array_equal(r.deg, want_d), (n, eps, min_pts)
            assert np.array_equal(r.labels, want_l), (n, eps, min_pts)


def test_sklearn_crosscheck_tie_free(orc):
    from sklearn.cluster import DBSCAN
    rng = np.random.default_rng(7)
    checked = 0
    for trial in range(12):
        n = int(rng.integers(50, 700))
        d = int(rng.choice([2, 3, 5]))
        X = random_instance(rng, n, d, "blobs", spread=0.04)
        D = pairwise_sq(X)
        eps = float(np.quantile(np.sqrt(D[np.triu_indices(n, 1)]), rng.uniform(0.002, 0.05)))
        eps = eps * (1 + 1e-7)
        if np.min(np.abs(D - eps * eps)) < 1e-9 * eps * eps:
            continue  # not tie-free
        for min_pts in [1, 3, 6]:
            r = orc.dbscan(X, eps, min_pts, exhaustive=True)
            sk = DBSCAN(eps=eps, min_samples=min_pts + 1, algorithm="brute").fit(X.astype(np.float64))
            core = np.zeros(n, bool)
            core[sk.core_sample_indices_] = True
            assert np.array_equal(core, r.deg.astype(np.int64) >= min_pts)
            assert np.array_equal(sk.labels_ == -1, r.labels == -1)
            # the core partition is the same up to renaming
            pairs = set(zip(sk.labels_[core].tolist(), r.labels[core].tolist()))
            assert len(pairs) == len(set(sk.labels_[core])) == len(set(r.labels[core]))
            # each border's cluster is one it is adjacent to
            adj = (D <= eps * eps) & ~np.eye(n, dtype=bool)
            for b in np.nonzero(~core & (r.labels != -1))[0]:
                assert r.labels[b] in set(r.labels[np.nonzero(adj[b] & core)[0]].tolist())
            checked += 1
    assert checked >= 20
