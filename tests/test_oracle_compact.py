"""Pins of the oracle's label compaction: hand cases, and agreement with
numpy's sorted-unique inverse on every labelling the clustering produces."""
import numpy as np

from paper_2006_06743_amd import workloads as wl


def test_hand_cases(orc):
    out, k = orc.compact_labels(np.array([0, 0, -1, 3, 3, 0, 6, -1, 3], np.int32))
    assert k == 3
    assert out.tolist() == [0, 0, -1, 1, 1, 0, 2, -1, 1]
    out, k = orc.compact_labels(np.zeros(0, np.int32))
    assert k == 0 and out.size == 0
    out, k = orc.compact_labels(np.array([-1, -1], np.int32))
    assert k == 0 and out.tolist() == [-1, -1]
    # entries that name no root (out of range, or a non-root index) become -1
    out, k = orc.compact_labels(np.array([0, 7, 0, 1, -5, 5], np.int32))
    assert k == 2 and out.tolist() == [0, -1, 0, -1, -1, 1]


def test_matches_unique_inverse_on_clusterings(orc):
    rng = np.random.default_rng(4242)
    for trial in range(6):
        X = wl.random_instance(rng, 3000, 2, "blobs", spread=0.03)
        r = orc.dbscan(X, 0.02, 3, int(rng.integers(0, 2**63)), s=0.05)
        out, k = orc.compact_labels(r.labels)
        clustered = r.labels >= 0
        u, inv = np.unique(r.labels[clustered], return_inverse=True)
        assert k == u.size == r.n_clusters
        assert np.array_equal(out[clustered], inv.astype(np.int32))
        assert np.all(out[~clustered] == -1)
