"""Pins of the oracle's sampling step over a source range and of its grid
sweep (Algorithm 1, sampling step; Section 5 tunes eps over a grid).

`oracle.degrees(X, m, eps, seed, i0, i1)` adds the symmetrised degrees that
the samples of sources [i0, i1) contribute. It is pinned by
  - the whole range against the whole method's degrees and counters;
  - additivity: the degrees of a split range sum to the whole;
  - the closed form with every pair accepted, restricted to a range:
    deg[i] = [i0 <= i < i1] (m - self_i) + #{samples of sources in the range
    that land on i}, the partners drawn with the sampler pinned against
    rocRAND and numpy elsewhere.
`oracle.sweep` is pinned against one `oracle.dbscan` run per grid point.
"""
import numpy as np
import pytest

from paper_2006_06743_amd.workloads import random_instance


def _instance(trial):
    """A small seeded point set with an eps that accepts a fair share of
    slots, a sampler seed and m."""
    rng = np.random.default_rng(1000 + trial)
    n = int(rng.integers(30, 400))
    d = int(rng.integers(1, 6))
    kind = ("blobs", "grid", "uniform", "dupes")[trial % 4]
    X = random_instance(rng, n, d, kind)
    eps = {"grid": 3.0, "blobs": 0.08, "uniform": 0.3, "dupes": 0.05}[kind] * (1 + 0.1 * d)
    return X, float(eps), int(rng.integers(0, 2**63)), int(rng.integers(1, 40))


def _draws(orc, seed, n, m, i0, i1):
    return np.array([[orc.partner(seed, n, i, t) for t in range(m)] for i in range(i0, i1)],
                    np.int64).reshape(i1 - i0, m)


@pytest.mark.parametrize("trial", range(4))
def test_full_range_equals_whole_method(orc, trial):
    X, eps, seed, m = _instance(trial)
    n = X.shape[0]
    deg, slots, self_pairs, acc = orc.degrees(X, m, eps, seed, 0, n)
    r = orc.dbscan(X, eps, 3, seed, m=m)
    assert np.array_equal(deg, r.deg)
    assert (slots, self_pairs, acc) == (r.slots, r.self_pairs, r.accepted)
    assert int(deg.sum()) == 2 * acc


@pytest.mark.parametrize("trial", range(3))
def test_split_ranges_add_up(orc, trial):
    X, eps, seed, m = _instance(trial + 4)
    n = X.shape[0]
    whole, slots, self_pairs, acc = orc.degrees(X, m, eps, seed, 0, n)
    rng = np.random.default_rng(trial)
    for cuts in ([0], [n], [1], [n - 1], sorted(rng.integers(0, n + 1, 3).tolist())):
        edges = [0] + list(cuts) + [n]
        total = np.zeros(n, np.uint32)
        counts = np.zeros(3, np.int64)
        for a, b in zip(edges[:-1], edges[1:]):
            _, s1, s2, s3 = orc.degrees(X, m, eps, seed, a, b, deg=total)
            counts += (s1, s2, s3)
        assert np.array_equal(total, whole)
        assert tuple(counts) == (slots, self_pairs, acc)


def test_range_closed_form_with_every_pair_accepted(orc):
    rng = np.random.default_rng(8)
    for n, m, seed, i0, i1 in [(1, 5, 0, 0, 1), (2, 9, 1, 1, 2), (37, 13, 2, 5, 30),
                               (300, 7, 3, 0, 151), (300, 7, 3, 151, 300),
                               (64, 64, 2**63 + 5, 10, 11), (50, 3, 7, 20, 20)]:
        X = rng.normal(size=(n, 3)).astype(np.float32)
        deg, slots, self_pairs, acc = orc.degrees(X, m, 1e30, seed, i0, i1)
        js = _draws(orc, seed, n, m, i0, i1)
        src = np.arange(i0, i1)[:, None]
        self_i = (js == src).sum(1)
        want = np.zeros(n, np.int64)
        want[i0:i1] += m - self_i
        np.add.at(want, js[js != src], 1)
        assert np.array_equal(deg.astype(np.int64), want)
        assert slots == (i1 - i0) * m and self_pairs == int(self_i.sum())
        assert acc == (i1 - i0) * m - int(self_i.sum())


def test_range_rejects_bad_bounds(orc):
    X = np.zeros((5, 2), np.float32)
    for i0, i1 in [(-1, 3), (2, 1), (0, 6)]:
        with pytest.raises(orc.OracleError):
            orc.degrees(X, 3, 1.0, 0, i0, i1)


@pytest.mark.parametrize("out_degree", [False, True])
@pytest.mark.parametrize("trial", range(3))
def test_sweep_equals_one_run_per_grid_point(orc, trial, out_degree):
    X, eps, seed, m = _instance(trial + 8)
    rng = np.random.default_rng(trial)
    # unsorted grid with a repeated value and eps = 0 (duplicates only)
    grid = np.array([eps, eps * 0.5, 0.0, eps * 1.7, eps, eps * 0.9])
    mps = [-1, 1, 2, int(rng.integers(3, 8))]
    labels, degs, st = orc.sweep(X, grid, mps, seed, m=m, out_degree=out_degree)
    for k, e in enumerate(grid):
        for p, mp in enumerate(mps):
            r = orc.dbscan(X, float(e), mp, seed, m=m, out_degree=out_degree)
            assert np.array_equal(labels[p, k], r.labels), (k, p)
            assert np.array_equal(degs[k], r.deg), k
            assert tuple(int(v) for v in st[p, k, :6]) == (
                r.slots, r.self_pairs, r.accepted, r.n_core, r.n_clusters, r.n_noise)


def test_sweep_on_a_log_spaced_grid(orc):
    """The sweep workload's shape of grid (log-spaced eps, MinPts doubling)
    on a small mixture, against one run per point."""
    rng = np.random.default_rng(11)
    X = np.concatenate([rng.normal(c, 0.4, size=(150, 4)) for c in (0.0, 3.0, 6.0)])
    X = X[rng.permutation(len(X))].astype(np.float32)
    grid = 0.2 * 3.0 ** (np.arange(8) / 7.0)
    mps = [2, 4, 8, 16]
    labels, degs, _ = orc.sweep(X, grid, mps, 4, s=0.05)
    for k, e in enumerate(grid):
        for p, mp in enumerate(mps):
            r = orc.dbscan(X, float(e), mp, 4, s=0.05)
            assert np.array_equal(labels[p, k], r.labels)
            assert np.array_equal(degs[k], r.deg)


def test_sweep_rejects_bad_grids(orc):
    X = np.zeros((4, 2), np.float32)
    for grid in ([1.0, -0.5], [float("nan")], [float("inf")]):
        with pytest.raises(orc.OracleError):
            orc.sweep(X, grid, [2], 0, m=2)
