"""Textbook O(n^2) DBSCAN written independently of the oracle (numpy, BFS).

Used only at full sampling (every pair queried), where SNG-DBSCAN reduces to
DBSCAN on the full eps-neighbourhood graph (Section 3: the method is a sampled
version of brute force). Labels use the same canonical form: a cluster is
named by its smallest core index; a non-core point takes the cluster of its
smallest-index core neighbour; -1 is noise. Degrees exclude the point itself.
"""
from collections import deque

import numpy as np


def pairwise_sq(X: np.ndarray) -> np.ndarray:
    X = X.astype(np.float64)
    D = np.zeros((X.shape[0], X.shape[0]))
    for k in range(X.shape[1]):
        diff = X[:, None, k] - X[None, :, k]
        D += diff * diff
    return D


def dbscan_bruteforce(X: np.ndarray, eps: float, min_pts: int):
    D = pairwise_sq(X)
    return dbscan_adjacency(D <= eps * eps, min_pts)


def dbscan_adjacency(adj: np.ndarray, min_pts: int):
    """DBSCAN on a given symmetric boolean neighbourhood matrix (the diagonal
    is ignored)."""
    adj = np.array(adj, dtype=bool)
    n = adj.shape[0]
    np.fill_diagonal(adj, False)
    deg = adj.sum(axis=1)
    core = deg >= min_pts
    labels = np.full(n, -1, np.int64)
    for c in range(n):
        if not core[c] or labels[c] != -1:
            continue
        labels[c] = c
        q = deque([c])
        while q:
            u = q.popleft()
            for v in np.nonzero(adj[u] & core)[0]:
                if labels[v] == -1:
                    labels[v] = c
                    q.append(v)
    for b in range(n):
        if core[b]:
            continue
        nb = np.nonzero(adj[b] & core)[0]
        labels[b] = labels[nb.min()] if nb.size else -1
    return labels.astype(np.int32), deg.astype(np.uint32), adj
