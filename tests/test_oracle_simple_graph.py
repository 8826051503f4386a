"""Pins for the simple-graph degree mode of the oracle: the sampled graph of
Algorithm 1 read as a simple graph, so a point's degree is its number of
distinct accepted neighbours, whichever endpoint sampled the pair and however
often. Pinned by set arithmetic on the sampler's partners (with every slot
accepted), a brute-force DBSCAN on the sampled simple graph, and invariants
against the multigraph and out-degree modes."""
import numpy as np

from bruteforce import dbscan_adjacency


def _partners(orc, seed, n, m):
    return np.array([[orc.partner(seed, n, i, t) for t in range(m)] for i in range(n)],
                    np.int64).reshape(n, m)


def test_every_slot_accepted_closed_form(orc):
    """deg[i] = |({S(i,t)} u {j : i in S(j,.)}) \\ {i}| when every slot is an edge."""
    rng = np.random.default_rng(21)
    for n, m, seed in [(2, 5, 0), (7, 3, 1), (40, 12, 2), (150, 30, 2**63 + 9)]:
        X = rng.normal(size=(n, 3)).astype(np.float32)
        r = orc.dbscan(X, 1e30, 1, seed, m=m, simple_graph=True)
        js = _partners(orc, seed, n, m)
        nb = [set() for _ in range(n)]
        for i in range(n):
            for j in js[i]:
                if j != i:
                    nb[i].add(int(j))
                    nb[int(j)].add(i)
        assert r.deg.tolist() == [len(s) for s in nb]


def test_two_points_count_once(orc):
    X = np.array([[0, 0], [1, 0]], np.float32)
    r = orc.dbscan(X, 2.0, 1, 3, m=9, simple_graph=True)
    assert r.deg.tolist() == [1, 1] and r.labels.tolist() == [0, 0]
    multi = orc.dbscan(X, 2.0, 1, 3, m=9)
    assert multi.deg.sum() > 2  # the multigraph counts every sampled slot
    r = orc.dbscan(X, 0.5, 1, 3, m=9, simple_graph=True)
    assert r.deg.tolist() == [0, 0]


def test_matches_bruteforce_on_the_sampled_simple_graph(orc):
    rng = np.random.default_rng(22)
    for n, d, m, seed, eps, mp in [(120, 2, 20, 4, 0.3, 3), (200, 3, 9, 5, 0.5, 4),
                                   (90, 2, 60, 6, 0.2, 6), (160, 1, 15, 7, 0.05, 2)]:
        X = rng.uniform(size=(n, d)).astype(np.float32)
        js = _partners(orc, seed, n, m)
        adj = np.zeros((n, n), bool)
        for i in range(n):
            for j in js[i]:
                if j != i and orc.sqdist(X, i, j) <= eps * eps:
                    adj[i, j] = adj[j, i] = True
        want_labels, want_deg, _ = dbscan_adjacency(adj, mp)
        r = orc.dbscan(X, eps, mp, seed, m=m, simple_graph=True)
        assert np.array_equal(r.deg, want_deg) and np.array_equal(r.labels, want_labels)


def test_invariants_against_the_other_modes(orc):
    rng = np.random.default_rng(23)
    X = rng.normal(size=(600, 4)).astype(np.float32)
    for seed, m, eps in [(1, 40, 1.0), (2, 200, 0.7)]:
        simple = orc.dbscan(X, eps, 0, seed, m=m, simple_graph=True)
        multi = orc.dbscan(X, eps, 0, seed, m=m)
        out = orc.dbscan(X, eps, 0, seed, m=m, out_degree=True)
        assert np.all(simple.deg <= multi.deg) and np.all(simple.deg <= 599)
        # a point's distinct own partners never exceed its simple degree
        js = _partners(orc, seed, 600, m)
        own = np.array([len({int(j) for j in js[i]
                             if j != i and orc.sqdist(X, i, int(j)) <= eps * eps})
                        for i in range(600)])
        assert np.all(own <= simple.deg) and np.all(own <= out.deg)
        assert int(simple.deg.sum()) % 2 == 0
        # MinPts <= 0 makes every point core: the components are the same graph's
        assert np.array_equal(simple.labels, multi.labels)
        for mp in [3, 8]:
            s = orc.dbscan(X, eps, mp, seed, m=m, simple_graph=True)
            core = simple.deg >= mp
            assert s.n_core == int(core.sum())


def test_similarity_query_simple_graph(orc):
    rng = np.random.default_rng(24)
    X = rng.normal(size=(300, 5)).astype(np.float32)
    r = orc.dbscan_similarity(X, orc.COSINE, 0.5, 2, seed=3, m=30, simple_graph=True)
    js = _partners(orc, 3, 300, 30)
    adj = np.zeros((300, 300), bool)
    for i in range(300):
        for j in js[i]:
            if j != i and orc.cosine(X, i, int(j)) >= 0.5:
                adj[i, j] = adj[j, i] = True
    want_labels, want_deg, _ = dbscan_adjacency(adj, 2)
    assert np.array_equal(r.deg, want_deg) and np.array_equal(r.labels, want_labels)
