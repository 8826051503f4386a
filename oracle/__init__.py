"""SNG-DBSCAN CPU oracle -- TEST INFRASTRUCTURE ONLY.

Thin ctypes view of ``libsng_oracle.so`` (plain C, binary64, written from
Algorithm 1 of the paper; see ``sng_oracle.h`` for the readings it fixes).
Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this module. The GPU library never links or calls it.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import build as _build

_lib = None


def load() -> ctypes.CDLL:
    """Load the oracle library, building it first only if nothing is built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    P = ctypes.c_void_p
    i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    lib.sng_oracle_philox4x32_10.argtypes = [P, P, P]
    lib.sng_oracle_philox4x32_10.restype = None
    lib.sng_oracle_philox4x64_10.argtypes = [P, P, P]
    lib.sng_oracle_philox4x64_10.restype = None
    lib.sng_oracle_samples_per_point.argtypes = [dbl, i64]
    lib.sng_oracle_samples_per_point.restype = i64
    lib.sng_oracle_partner.argtypes = [u64, i64, i64, i64]
    lib.sng_oracle_partner.restype = ctypes.c_uint32
    lib.sng_oracle_sqdist.argtypes = [P, i64, i32, i64, i64]
    lib.sng_oracle_sqdist.restype = dbl
    lib.sng_oracle_degrees_range.argtypes = [P, i64, i32, i64, i64, dbl, u64, i64, i64, P, P]
    lib.sng_oracle_degrees_range.restype = ctypes.c_int
    lib.sng_oracle_slot_sqdist.argtypes = [P, i64, i32, i64, i64, u64, i64, i64, P]
    lib.sng_oracle_slot_sqdist.restype = ctypes.c_int
    lib.sng_oracle_dbscan.argtypes = [P, i64, i32, i64, i64, dbl, i32, u64, i32, P, P, P]
    lib.sng_oracle_dbscan.restype = ctypes.c_int
    lib.sng_oracle_dot.argtypes = [P, i64, i32, i64, i64]
    lib.sng_oracle_dot.restype = dbl
    lib.sng_oracle_cosine.argtypes = [P, i64, i32, i64, i64]
    lib.sng_oracle_cosine.restype = dbl
    lib.sng_oracle_dbscan_similarity.argtypes = [P, i64, i32, i64, i64, i32, dbl, i32, u64, i32,
                                                 P, P, P]
    lib.sng_oracle_dbscan_similarity.restype = ctypes.c_int
    lib.sng_oracle_sweep.argtypes = [P, i64, i32, i64, i64, P, i32, P, i32, u64, i32, P, P, P]
    lib.sng_oracle_sweep.restype = ctypes.c_int
    lib.sng_oracle_graph.argtypes = [i64, P, i64, i32, P, P, P]
    lib.sng_oracle_graph.restype = ctypes.c_int
    _lib = lib
    return lib


def set_threads(n: int) -> int:
    """Sets the oracle's OpenMP thread count (omp_set_num_threads of the
    OpenMP runtime it links) and returns omp_get_max_threads() after it."""
    load()
    gomp = ctypes.CDLL("libgomp.so.1")
    gomp.omp_set_num_threads(ctypes.c_int(int(n)))
    return int(gomp.omp_get_max_threads())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError("%s failed with code %d" % (what, rc))


@dataclass
class Result:
    labels: np.ndarray   # int32 [n]
    deg: np.ndarray      # uint32 [n]
    slots: int
    self_pairs: int
    accepted: int
    n_core: int
    n_clusters: int
    n_noise: int


def _result(labels, deg, st) -> Result:
    return Result(labels, deg, int(st[0]), int(st[1]), int(st[2]), int(st[3]), int(st[4]),
                  int(st[5]))


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    load().sng_oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox4x64_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    load().sng_oracle_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def samples_per_point(s: float, n: int) -> int:
    return int(load().sng_oracle_samples_per_point(float(s), int(n)))


def partner(seed: int, n: int, i: int, t: int) -> int:
    return int(load().sng_oracle_partner(int(seed), int(n), int(i), int(t)))


def sqdist(X: np.ndarray, i: int, j: int) -> float:
    X = _rows(X)
    return float(load().sng_oracle_sqdist(_ptr(X), X.shape[1], X.shape[1], int(i), int(j)))


DOT, COSINE = 1, 2  # similarity kinds (edge when the similarity is >= tau)


def dot(X: np.ndarray, i: int, j: int) -> float:
    """<x_i, x_j> in binary64, coordinate order."""
    X = _rows(X)
    return float(load().sng_oracle_dot(_ptr(X), X.shape[1], X.shape[1], int(i), int(j)))


def cosine(X: np.ndarray, i: int, j: int) -> float:
    """<x_i, x_j> / (|x_i| |x_j|) in binary64 (NaN for a zero row)."""
    X = _rows(X)
    return float(load().sng_oracle_cosine(_ptr(X), X.shape[1], X.shape[1], int(i), int(j)))


def _rows(X: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise ValueError("X must be [n, d]")
    return X


def degrees(X: np.ndarray, m: int, eps: float, seed: int, i0: int = 0,
            i1: Optional[int] = None, deg: Optional[np.ndarray] = None):
    """Sampling step over sources [i0, i1): returns (deg, slots, self, accepted)."""
    X = _rows(X)
    n, d = X.shape
    i1 = n if i1 is None else i1
    if deg is None:
        deg = np.zeros(n, np.uint32)
    st = np.zeros(8, np.uint64)
    _check(load().sng_oracle_degrees_range(_ptr(X), n, d, d, int(m), float(eps), int(seed),
                                           int(i0), int(i1), _ptr(deg), _ptr(st)),
           "sng_oracle_degrees_range")
    return deg, int(st[0]), int(st[1]), int(st[2])


def slot_sqdist(X: np.ndarray, m: int, seed: int, i0: int = 0, i1: Optional[int] = None):
    X = _rows(X)
    n, d = X.shape
    i1 = n if i1 is None else i1
    out = np.empty((i1 - i0) * int(m), np.float64)
    _check(load().sng_oracle_slot_sqdist(_ptr(X), n, d, d, int(m), int(seed), int(i0), int(i1),
                                         _ptr(out)), "sng_oracle_slot_sqdist")
    return out.reshape(i1 - i0, int(m))


def _mode(exhaustive: bool, out_degree: bool, simple_graph: bool) -> int:
    if exhaustive + out_degree + simple_graph > 1:
        raise OracleError("exhaustive, out_degree and simple_graph exclude each other")
    return 1 if exhaustive else (2 if out_degree else (3 if simple_graph else 0))


def dbscan(X: np.ndarray, eps: float, min_pts: int, seed: int = 0, s: Optional[float] = None,
           m: Optional[int] = None, exhaustive: bool = False,
           out_degree: bool = False, simple_graph: bool = False) -> Result:
    """SNG-DBSCAN (Algorithm 1). Give ``s`` (m = ceil(s*n)) or ``m``;
    ``exhaustive=True`` uses the full eps-neighbourhood graph instead;
    ``out_degree=True`` counts only a point's own accepted samples in its
    degree (Lemma 2, Section 4.1); ``simple_graph=True`` counts distinct
    accepted neighbours (each sampled pair once)."""
    X = _rows(X)
    n, d = X.shape
    if not exhaustive:
        if m is None:
            m = samples_per_point(s, n)
            if m < 0:
                raise OracleError("invalid sampling rate")
    labels = np.empty(n, np.int32)
    deg = np.zeros(n, np.uint32)
    st = np.zeros(8, np.uint64)
    _check(load().sng_oracle_dbscan(_ptr(X), n, d, d, int(m or 0), float(eps), int(min_pts),
                                    int(seed), _mode(exhaustive, out_degree, simple_graph),
                                    _ptr(labels), _ptr(deg),
                                    _ptr(st)), "sng_oracle_dbscan")
    return _result(labels, deg, st)


def dbscan_similarity(X: np.ndarray, kind: int, tau: float, min_pts: int, seed: int = 0,
                      s: Optional[float] = None, m: Optional[int] = None,
                      exhaustive: bool = False, out_degree: bool = False,
                      simple_graph: bool = False) -> Result:
    """SNG-DBSCAN with a similarity query instead of the distance (Section 1):
    an edge when the dot product (kind DOT) or the cosine (kind COSINE) of the
    pair is >= tau. Sampling, modes and post-processing as in ``dbscan``."""
    X = _rows(X)
    n, d = X.shape
    if not exhaustive and m is None:
        m = samples_per_point(s, n)
        if m < 0:
            raise OracleError("invalid sampling rate")
    labels = np.empty(n, np.int32)
    deg = np.zeros(n, np.uint32)
    st = np.zeros(8, np.uint64)
    _check(load().sng_oracle_dbscan_similarity(_ptr(X), n, d, d, int(m or 0), int(kind),
                                               float(tau), int(min_pts), int(seed),
                                               _mode(exhaustive, out_degree, simple_graph),
                                               _ptr(labels), _ptr(deg), _ptr(st)),
           "sng_oracle_dbscan_similarity")
    return _result(labels, deg, st)


def graph(n: int, edges, min_pts: int) -> Result:
    """Post-processing only, on an explicit list of accepted pairs."""
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64).reshape(-1, 2))
    labels = np.empty(n, np.int32)
    deg = np.zeros(n, np.uint32)
    st = np.zeros(8, np.uint64)
    _check(load().sng_oracle_graph(int(n), _ptr(e), e.shape[0], int(min_pts), _ptr(labels),
                                   _ptr(deg), _ptr(st)), "sng_oracle_graph")
    return _result(labels, deg, st)


def sweep(X: np.ndarray, eps_grid, min_pts_grid, seed: int, s: Optional[float] = None,
          m: Optional[int] = None, out_degree: bool = False):
    """Every (eps, MinPts) pair of a grid (Section 5 tunes eps over a grid),
    each equal to ``dbscan(X, eps, MinPts, seed, ...)``: one sampling step at
    the largest eps, then each grid point's edges taken from its accepted
    pairs by the single run's own test. Returns labels [P][K][n], degrees
    [K][n] and per-point stats [P][K][8]."""
    X = _rows(X)
    n, d = X.shape
    if m is None:
        m = samples_per_point(s, n)
        if m < 0:
            raise OracleError("invalid sampling rate")
    e = np.ascontiguousarray(eps_grid, dtype=np.float64).ravel()
    mp = np.ascontiguousarray(min_pts_grid, dtype=np.int32).ravel()
    K, P = e.size, mp.size
    labels = np.empty((P, K, n), np.int32)
    degs = np.empty((K, n), np.uint32)
    st = np.zeros((P, K, 8), np.uint64)
    _check(load().sng_oracle_sweep(_ptr(X), n, d, d, int(m), _ptr(e), K, _ptr(mp), P,
                                   int(seed), 2 if out_degree else 0, _ptr(labels), _ptr(degs),
                                   _ptr(st)), "sng_oracle_sweep")
    return labels, degs, st


def compact_labels(labels) -> tuple[np.ndarray, int]:
    """Clusters renamed 0..k-1 in increasing order of their root (the method
    fixes clusters only up to a renaming: Section 4.1, Theorem 1). A root is
    an r with labels[r] == r; an entry that is neither -1 nor a root's index
    becomes -1. Returns (int32 [n], k)."""
    L = np.asarray(labels, np.int64).ravel()
    n = L.size
    idx = np.arange(n)
    roots = idx[L == idx]  # ascending
    rank = np.full(n, -1, np.int64)
    rank[roots] = np.arange(roots.size)
    out = np.full(n, -1, np.int32)
    ok = (L >= 0) & (L < n)
    out[ok] = rank[L[ok]]
    return out, int(roots.size)
