"""SNG-DBSCAN on AMD Instinct MI355X (gfx950).

Python binding of libsng.so: argument marshalling only. Every step of the
method runs in the library's HIP kernels; PyTorch supplies device memory and
the current stream. The C ABI is documented in include/sng.h.

    labels, degrees = dbscan(X, s, eps, min_pts, seed)     # X: cuda float32 [n, d]
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import (SNG_BF16, SNG_FP16, SNG_FP32, SNG_SIM_COSINE, SNG_SIM_DOT, SNGError, check,
                   sng_config, sng_stats)

__all__ = ["dbscan", "dbscan_noalloc", "dbscan_lowp", "dbscan_similarity", "degrees", "sample", "cluster",
           "compact_labels", "similarity_workspace_size", "SNG_SIM_DOT", "SNG_SIM_COSINE",
           "autotune", "autotune_lookup", "autotune_clear", "autotune_save", "autotune_load",
           "autotune_hook", "autotune_lowp", "autotune_batch",
           "graph_labels", "sweep", "batch", "BatchPlan",
           "samples_per_point", "Config", "Stats", "SNGError", "SNG_FP32", "SNG_BF16",
           "SNG_FP16", "load"]


def load():
    """Loads libsng.so (raises ImportError if it is not built)."""
    return _lib.load()


@dataclass
class Config:
    lanes_per_pair: int = 0
    chunks_per_wave: int = 0
    stage_lds: int = 0
    prefetch: int = 0
    schedule: int = 0  # 0 auto, 1 direct gathers, 2 partner-block (L2 reuse)
    reuse_sample: int = 0  # 1: evaluate the sample that sample() left in the workspace
    out_degree: int = 0    # 1: a point's degree counts only its own accepted samples
    simple_graph: int = 0  # 1: a point's degree counts its distinct accepted neighbours
    mfma_waves: int = 0    # mixed form: wavefronts per block of the MFMA pass (1, 2, 4)
    mfma_ksteps: int = 0   # mixed form: 32-wide K-steps loaded together (4, 8, 16)
    hook_blocks: int = 0   # post-processing: grid of the hook launch (256..65536)

    def c(self):
        return ctypes.byref(sng_config(self.lanes_per_pair, self.chunks_per_wave,
                                       self.stage_lds, self.prefetch, self.schedule,
                                       self.reuse_sample, self.out_degree, self.simple_graph,
                                       self.mfma_waves, self.mfma_ksteps, self.hook_blocks))


@dataclass
class Stats:
    slots: int
    self_pairs: int
    accepted: int
    rechecked: int
    n_core: int
    n_clusters: int
    n_noise: int
    overflow: int
    band_rel: float
    filter_gamma: float = 0.0
    filter_r_max: float = 0.0
    filter_r_mean: float = 0.0
    filter_rel_width: float = 0.0


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def _rows(X: torch.Tensor):
    """(n, d, row stride) of a CUDA float32 matrix with unit column stride
    (strides of empty or single-row matrices are irrelevant)."""
    if not X.is_cuda or X.dtype != torch.float32 or X.dim() != 2:
        raise ValueError("X must be a CUDA float32 tensor [n, d]")
    n, d = X.shape
    if n > 0 and d > 1 and X.stride(1) != 1:
        raise ValueError("X must have unit column stride")
    return n, d, X.stride(0) if n > 1 else d


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _cfg(cfg: Optional[Config]):
    return cfg.c() if cfg is not None else None


def _ws_flags(cfg: Optional[Config]) -> int:
    """Workspace-size flags a configuration needs (the simple-graph table)."""
    return _lib.SNG_WS_SIMPLE_GRAPH if cfg is not None and cfg.simple_graph else 0


def samples_per_point(s: float, n: int) -> int:
    m = ctypes.c_int64()
    check(_lib.load().sng_samples_per_point(float(s), int(n), ctypes.byref(m)),
          "sng_samples_per_point")
    return m.value


def workspace_size(n: int, d: int, m: int, prec: int = SNG_FP32) -> int:
    b = ctypes.c_size_t()
    check(_lib.load().sng_workspace_size(int(n), int(d), int(m), int(prec), ctypes.byref(b)),
          "sng_workspace_size")
    return b.value


def stats(ws: torch.Tensor, index: int = 0) -> Stats:
    """Counters of the last call that used workspace `ws` (waits for its stream)."""
    st = sng_stats()
    rc = _lib.load().sng_stats_read(ws.data_ptr(), int(index), ctypes.byref(st), _stream(ws))
    if rc not in (_lib.SNG_OK, _lib.SNG_EOVERFLOW):
        check(rc, "sng_stats_read")
    return Stats(st.slots, st.self_pairs, st.accepted, st.rechecked, st.n_core, st.n_clusters,
                 st.n_noise, st.overflow, st.band_rel, st.filter_gamma, st.filter_r_max,
                 st.filter_r_mean, st.filter_rel_width)


def lowp_bound(ws: torch.Tensor) -> dict:
    """The mixed form's stated filter bound after a dbscan_lowp call on ws,
    with the fraction of slots it sent to the binary64 recheck."""
    st = stats(ws)
    return {"filter_gamma": st.filter_gamma, "r_max": st.filter_r_max,
            "r_mean": st.filter_r_mean, "rel_width_at_eps": st.filter_rel_width,
            "recheck_fraction": st.rechecked / max(1, st.slots)}


def degrees(X: torch.Tensor, m: int, eps: float, seed: int, cfg: Optional[Config] = None,
            out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None):
    """Sampling step only: symmetrised degrees (int32 tensor holding u32)."""
    n, d, ld = _rows(X)
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=X.device)
    if ws is None:
        ws = _ws(workspace_size(n, d, m, SNG_FP32 | _ws_flags(cfg)), X.device)
    check(_lib.load().sng_degrees(X.data_ptr(), n, d, ld, int(m), float(eps), int(seed),
                                  out.data_ptr(), ws.data_ptr(), ws.numel(), _cfg(cfg),
                                  _stream(X)), "sng_degrees")
    return out, ws


def sample(n: int, d: int, m: int, seed: int, ws: torch.Tensor):
    """Sampling step alone: draws every slot's partner and keeps the slots
    sorted by partner block in ws, for degrees()/dbscan() calls with
    Config(reuse_sample=1). ws: a workspace of workspace_size(n, d, m)."""
    check(_lib.load().sng_sample(int(n), int(d), int(m), int(seed), ws.data_ptr(), ws.numel(),
                                 _stream(ws)), "sng_sample")
    return ws


def _config_of(c) -> Config:
    return Config(c.lanes_per_pair, c.chunks_per_wave, c.stage_lds, c.prefetch, c.schedule,
                  c.reuse_sample, c.out_degree, c.simple_graph, c.mfma_waves, c.mfma_ksteps,
                  c.hook_blocks)


def autotune(X: torch.Tensor, m: int, eps: float, seed: int, trials: int = 2,
             ws: Optional[torch.Tensor] = None):
    """Times the launch shapes and schedules of the sampled-distance pass on X
    and caches the fastest for calls without a config. Returns
    (Config, mean ms, candidates timed)."""
    n, d, ld = _rows(X)
    if ws is None:
        ws = _ws(workspace_size(n, d, m), X.device)
    best = sng_config()
    ms = ctypes.c_float()
    tried = ctypes.c_int32()
    check(_lib.load().sng_autotune(X.data_ptr() if n else None, n, d, ld, int(m), float(eps),
                                   int(seed), ws.data_ptr(), ws.numel(), int(trials),
                                   ctypes.byref(best), ctypes.byref(ms), ctypes.byref(tried),
                                   _stream(X)), "sng_autotune")
    return _config_of(best), ms.value, tried.value


def autotune_lookup(X: torch.Tensor, m: int) -> Optional[Config]:
    """The cached tuned config for X's shape class, or None."""
    n, d, ld = _rows(X)
    out = sng_config()
    rc = _lib.load().sng_autotune_lookup(X.data_ptr() if n else None, n, d, ld, int(m),
                                         ctypes.byref(out))
    if rc == _lib.SNG_ENOTIMPL:
        return None
    check(rc, "sng_autotune_lookup")
    return _config_of(out)


def autotune_clear():
    check(_lib.load().sng_autotune_clear(), "sng_autotune_clear")


def autotune_save(path: str):
    """Writes the autotune cache to a text file."""
    check(_lib.load().sng_autotune_save(os.fsencode(path)), "sng_autotune_save")


def autotune_load(path: str):
    """Merges a file written by autotune_save into the autotune cache."""
    check(_lib.load().sng_autotune_load(os.fsencode(path)), "sng_autotune_load")


def autotune_hook(X: torch.Tensor, m: int, eps: float, seed: int, min_pts: int,
                  deg: torch.Tensor, ws: torch.Tensor, trials: int = 2,
                  labels: Optional[torch.Tensor] = None):
    """Times the hook launch's grid on the post-processing that a prior
    degrees() call on ws prepared, caches the fastest for the plain form's
    shape class. Returns (Config, mean ms, candidates timed, labels)."""
    n, d, ld = _rows(X)
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    best = sng_config()
    ms = ctypes.c_float()
    tried = ctypes.c_int32()
    check(_lib.load().sng_autotune_hook(X.data_ptr(), n, d, ld, int(m), float(eps), int(seed),
                                        int(min_pts), deg.data_ptr(), labels.data_ptr(),
                                        ws.data_ptr(), ws.numel(), int(trials),
                                        ctypes.byref(best), ctypes.byref(ms),
                                        ctypes.byref(tried), _stream(X)), "sng_autotune_hook")
    return _config_of(best), ms.value, tried.value, labels


def cluster(X: torch.Tensor, m: int, eps: float, seed: int, min_pts: int, deg: torch.Tensor,
            ws: torch.Tensor, labels: Optional[torch.Tensor] = None):
    """Post-processing continuing from the accept bits a prior degrees() call left in ws."""
    n, d, ld = _rows(X)
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    check(_lib.load().sng_cluster(X.data_ptr(), n, d, ld, int(m), float(eps), int(seed),
                                  int(min_pts), deg.data_ptr(), labels.data_ptr(), ws.data_ptr(),
                                  ws.numel(), _stream(X)), "sng_cluster")
    return labels


def dbscan(X: torch.Tensor, s: float, eps: float, min_pts: int, seed: int,
           cfg: Optional[Config] = None, want_degrees: bool = True,
           labels: Optional[torch.Tensor] = None, degrees_out: Optional[torch.Tensor] = None,
           ws: Optional[torch.Tensor] = None):
    """SNG-DBSCAN (Algorithm 1): returns (labels int32, degrees int32-as-u32 or None, ws)."""
    n, d, ld = _rows(X)
    m = samples_per_point(s, n)
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    if want_degrees and degrees_out is None:
        degrees_out = torch.empty(n, dtype=torch.int32, device=X.device)
    if ws is None:
        ws = _ws(workspace_size(n, d, m, SNG_FP32 | _ws_flags(cfg)), X.device)
    check(_lib.load().sng_dbscan(X.data_ptr(), n, d, ld, float(s), float(eps), int(min_pts),
                                 int(seed), labels.data_ptr(),
                                 degrees_out.data_ptr() if degrees_out is not None else None,
                                 ws.data_ptr(), ws.numel(), _cfg(cfg), _stream(X)),
          "sng_dbscan")
    return labels, degrees_out, ws


def dbscan_noalloc(X: torch.Tensor, s: float, eps: float, min_pts: int, seed: int,
                   cfg: Optional[Config] = None, labels: Optional[torch.Tensor] = None,
                   degrees_out: Optional[torch.Tensor] = None):
    """sng_dbscan_noalloc: SNG-DBSCAN with the library's static device
    scratch array as workspace (the C call allocates nothing; outputs are
    allocated here when not given). Returns (labels, degrees or None)."""
    n, d, ld = _rows(X)
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    check(_lib.load().sng_dbscan_noalloc(X.data_ptr(), n, d, ld, float(s), float(eps),
                                         int(min_pts), int(seed), labels.data_ptr(),
                                         degrees_out.data_ptr() if degrees_out is not None
                                         else None, _cfg(cfg), _stream(X)),
          "sng_dbscan_noalloc")
    return labels, degrees_out


def similarity_workspace_size(n: int, d: int, m: int, kind: int, flags: int = 0) -> int:
    b = ctypes.c_size_t()
    check(_lib.load().sng_similarity_workspace_size(int(n), int(d), int(m), int(kind),
                                                    int(flags), ctypes.byref(b)),
          "sng_similarity_workspace_size")
    return b.value


def dbscan_similarity(X: torch.Tensor, s: float, kind: int, tau: float, min_pts: int, seed: int,
                      cfg: Optional[Config] = None, want_degrees: bool = True,
                      labels: Optional[torch.Tensor] = None,
                      degrees_out: Optional[torch.Tensor] = None,
                      ws: Optional[torch.Tensor] = None):
    """SNG-DBSCAN with a similarity query: an edge when the dot product
    (SNG_SIM_DOT) or the cosine (SNG_SIM_COSINE) of a sampled pair is >= tau.
    Returns (labels, degrees or None, ws)."""
    n, d, ld = _rows(X)
    m = samples_per_point(s, n)
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    if want_degrees and degrees_out is None:
        degrees_out = torch.empty(n, dtype=torch.int32, device=X.device)
    if ws is None:
        ws = _ws(similarity_workspace_size(n, d, m, kind, _ws_flags(cfg)), X.device)
    check(_lib.load().sng_dbscan_similarity(X.data_ptr(), n, d, ld, float(s), int(kind),
                                            float(tau), int(min_pts), int(seed),
                                            labels.data_ptr(),
                                            degrees_out.data_ptr() if degrees_out is not None
                                            else None,
                                            ws.data_ptr(), ws.numel(), _cfg(cfg), _stream(X)),
          "sng_dbscan_similarity")
    return labels, degrees_out, ws


def dbscan_lowp(X: torch.Tensor, X_lp: torch.Tensor, s: float, eps: float, min_pts: int,
                seed: int, prec: int = SNG_BF16, lp_scale: float = 1.0,
                cfg: Optional[Config] = None, ws: Optional[torch.Tensor] = None):
    """Mixed-precision form: X_lp holds bfloat16/float16 bits (int16/bf16/fp16 tensor)."""
    n, d, ld = _rows(X)
    if X_lp.element_size() != 2 or X_lp.dim() != 2 or X_lp.stride(1) != 1 or not X_lp.is_cuda:
        raise ValueError("X_lp must be a CUDA 16-bit tensor [n, >=d] with unit column stride")
    m = samples_per_point(s, n)
    labels = torch.empty(n, dtype=torch.int32, device=X.device)
    deg = torch.empty(n, dtype=torch.int32, device=X.device)
    if ws is None:
        ws = _ws(workspace_size(n, d, m, prec), X.device)
    check(_lib.load().sng_dbscan_lowp(X.data_ptr(), n, d, ld, X_lp.data_ptr(),
                                      X_lp.stride(0) if n > 0 else d, float(lp_scale), int(prec),
                                      float(s), float(eps), int(min_pts), int(seed),
                                      labels.data_ptr(), deg.data_ptr(), ws.data_ptr(),
                                      ws.numel(), _cfg(cfg), _stream(X)), "sng_dbscan_lowp")
    return labels, deg, ws


def autotune_lowp(X: torch.Tensor, X_lp: torch.Tensor, s: float, eps: float, min_pts: int,
                  seed: int, prec: int = SNG_BF16, lp_scale: float = 1.0, trials: int = 2,
                  ws: Optional[torch.Tensor] = None):
    """Times the mixed form's MFMA pass shapes (whole dbscan_lowp calls) and
    caches the fastest for its precision and shape class. Returns (Config,
    mean ms, candidates timed, labels, degrees)."""
    n, d, ld = _rows(X)
    m = samples_per_point(s, n)
    labels = torch.empty(n, dtype=torch.int32, device=X.device)
    deg = torch.empty(n, dtype=torch.int32, device=X.device)
    if ws is None:
        ws = _ws(workspace_size(n, d, m, prec), X.device)
    best = sng_config()
    ms = ctypes.c_float()
    tried = ctypes.c_int32()
    check(_lib.load().sng_autotune_lowp(X.data_ptr(), n, d, ld, X_lp.data_ptr(),
                                        X_lp.stride(0) if n > 0 else d, float(lp_scale),
                                        int(prec), float(s), float(eps), int(min_pts), int(seed),
                                        labels.data_ptr(), deg.data_ptr(), ws.data_ptr(),
                                        ws.numel(), int(trials), ctypes.byref(best),
                                        ctypes.byref(ms), ctypes.byref(tried), _stream(X)),
          "sng_autotune_lowp")
    return _config_of(best), ms.value, tried.value, labels, deg


def graph_labels(n: int, edges: torch.Tensor, min_pts: int, device=None):
    """Post-processing only on an explicit accepted-pair list (int32 [E, 2])."""
    dev = edges.device if edges.is_cuda else torch.device(device or "cuda")
    e = edges.to(device=dev, dtype=torch.int32).contiguous()
    b = ctypes.c_size_t()
    check(_lib.load().sng_graph_workspace_size(int(n), ctypes.byref(b)),
          "sng_graph_workspace_size")
    ws = _ws(b.value, dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    deg = torch.empty(n, dtype=torch.int32, device=dev)
    check(_lib.load().sng_graph_labels(int(n), e.data_ptr() if e.numel() else None,
                                       e.shape[0], int(min_pts), labels.data_ptr(),
                                       deg.data_ptr(), ws.data_ptr(), ws.numel(),
                                       torch.cuda.current_stream(dev).cuda_stream),
          "sng_graph_labels")
    return labels, deg, ws


def compact_labels(labels: torch.Tensor, out: Optional[torch.Tensor] = None):
    """Clusters renumbered 0..k-1 in increasing root order (noise stays -1):
    returns (out int32 [n], n_clusters int32 [1]), both on the device."""
    if not labels.is_cuda or labels.dtype != torch.int32 or labels.dim() != 1:
        raise ValueError("labels must be a 1-D int32 device tensor")
    lab = labels.contiguous()
    n = lab.numel()
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=lab.device)
    k = torch.empty(1, dtype=torch.int32, device=lab.device)
    check(_lib.load().sng_compact_labels(lab.data_ptr() if n else None, n,
                                         out.data_ptr() if n else None, k.data_ptr(),
                                         torch.cuda.current_stream(lab.device).cuda_stream),
          "sng_compact_labels")
    return out, k


def sweep(X: torch.Tensor, s: float, eps_grid: Sequence[float], min_pts_grid: Sequence[int],
          seed: int, want_degrees: bool = True, ws: Optional[torch.Tensor] = None,
          cfg: Optional[Config] = None):
    """All (eps, MinPts) pairs of a grid from one sampled-distance pass:
    labels [P][K][n] int32, degrees [K][n] (u32 bits) or None."""
    import numpy as np
    n, d, ld = _rows(X)
    m = samples_per_point(s, n)
    eps = np.ascontiguousarray(eps_grid, dtype=np.float64)
    mp = np.ascontiguousarray(min_pts_grid, dtype=np.int32)
    K, P = eps.size, mp.size
    b = ctypes.c_size_t()
    check(_lib.load().sng_sweep_workspace_size(n, d, m, K, P, ctypes.byref(b)),
          "sng_sweep_workspace_size")
    if ws is None:
        ws = _ws(b.value, X.device)
    labels = torch.empty((P, K, n), dtype=torch.int32, device=X.device)
    deg = torch.empty((K, n), dtype=torch.int32, device=X.device) if want_degrees else None
    check(_lib.load().sng_dbscan_sweep(X.data_ptr(), n, d, ld, float(s), eps.ctypes.data, K,
                                       mp.ctypes.data, P, int(seed), labels.data_ptr(),
                                       deg.data_ptr() if deg is not None else None,
                                       ws.data_ptr(), ws.numel(), _cfg(cfg), _stream(X)),
          "sng_dbscan_sweep")
    return labels, deg, ws


def _batch_args(Xs, s, eps, min_pts, seeds, labels, degs):
    import numpy as np
    count = len(Xs)
    d = Xs[0].shape[1]
    arr = lambda vals, dt: np.ascontiguousarray(vals, dtype=dt)
    xp = arr([x.data_ptr() for x in Xs], np.uint64)
    ns = arr([x.shape[0] for x in Xs], np.int64)
    lds = arr([x.stride(0) if x.shape[0] > 0 else d for x in Xs], np.int64)
    ss = arr(s, np.float64)
    es = arr(eps, np.float64)
    ms = arr(min_pts, np.int32)
    sd = arr(seeds, np.uint64)
    lp = arr([t.data_ptr() for t in labels], np.uint64)
    dp = arr([t.data_ptr() for t in degs], np.uint64)
    return count, d, (xp, ns, lds, ss, es, ms, sd, lp, dp)


def batch_workspace_size(ns, d, s) -> int:
    import numpy as np
    n_arr = np.ascontiguousarray(ns, dtype=np.int64)
    s_arr = np.ascontiguousarray(s, dtype=np.float64)
    b = ctypes.c_size_t()
    check(_lib.load().sng_batch_workspace_size(len(n_arr), n_arr.ctypes.data, int(d),
                                               s_arr.ctypes.data, ctypes.byref(b)),
          "sng_batch_workspace_size")
    return b.value


def batch(Xs, s, eps, min_pts, seeds, ws: Optional[torch.Tensor] = None):
    """Independent instances solved together; returns per-instance (labels, degrees)."""
    for x in Xs:
        _rows(x)
    dev = Xs[0].device
    labels = [torch.empty(x.shape[0], dtype=torch.int32, device=dev) for x in Xs]
    degs = [torch.empty(x.shape[0], dtype=torch.int32, device=dev) for x in Xs]
    count, d, a = _batch_args(Xs, s, eps, min_pts, seeds, labels, degs)
    if ws is None:
        ws = _ws(batch_workspace_size(a[1], d, a[3]), dev)
    xp, ns, lds, ss, es, ms, sd, lp, dp = a
    check(_lib.load().sng_dbscan_batch(count, xp.ctypes.data, ns.ctypes.data, d, lds.ctypes.data,
                                       ss.ctypes.data, es.ctypes.data, ms.ctypes.data,
                                       sd.ctypes.data, lp.ctypes.data, dp.ctypes.data,
                                       ws.data_ptr(), ws.numel(), _stream(Xs[0])),
          "sng_dbscan_batch")
    return labels, degs, ws


def autotune_batch(Xs, s, eps, min_pts, seeds, trials: int = 2,
                   ws: Optional[torch.Tensor] = None):
    """Times launch shapes of the batched pass on this batch and caches the
    fastest for its shape class. Returns (Config, mean ms, candidates timed,
    labels, degrees)."""
    for x in Xs:
        _rows(x)
    dev = Xs[0].device
    labels = [torch.empty(x.shape[0], dtype=torch.int32, device=dev) for x in Xs]
    degs = [torch.empty(x.shape[0], dtype=torch.int32, device=dev) for x in Xs]
    count, d, a = _batch_args(Xs, s, eps, min_pts, seeds, labels, degs)
    if ws is None:
        ws = _ws(batch_workspace_size(a[1], d, a[3]), dev)
    xp, ns, lds, ss, es, ms_, sd, lp, dp = a
    best = sng_config()
    ms = ctypes.c_float()
    tried = ctypes.c_int32()
    check(_lib.load().sng_autotune_batch(count, xp.ctypes.data, ns.ctypes.data, d,
                                         lds.ctypes.data, ss.ctypes.data, es.ctypes.data,
                                         ms_.ctypes.data, sd.ctypes.data, lp.ctypes.data,
                                         dp.ctypes.data, ws.data_ptr(), ws.numel(), int(trials),
                                         ctypes.byref(best), ctypes.byref(ms),
                                         ctypes.byref(tried), _stream(Xs[0])),
          "sng_autotune_batch")
    return _config_of(best), ms.value, tried.value, labels, degs


class BatchPlan:
    """A batch recorded once into a HIP graph and replayed by launch()."""

    def __init__(self, Xs, s, eps, min_pts, seeds):
        for x in Xs:
            _rows(x)
        dev = Xs[0].device
        self.Xs = list(Xs)
        self.labels = [torch.empty(x.shape[0], dtype=torch.int32, device=dev) for x in Xs]
        self.degrees = [torch.empty(x.shape[0], dtype=torch.int32, device=dev) for x in Xs]
        count, d, a = _batch_args(Xs, s, eps, min_pts, seeds, self.labels, self.degrees)
        self.ws = _ws(batch_workspace_size(a[1], d, a[3]), dev)
        xp, ns, lds, ss, es, ms, sd, lp, dp = a
        self._plan = ctypes.c_void_p()
        check(_lib.load().sng_batch_plan_create(
            count, xp.ctypes.data, ns.ctypes.data, d, lds.ctypes.data, ss.ctypes.data,
            es.ctypes.data, ms.ctypes.data, sd.ctypes.data, lp.ctypes.data, dp.ctypes.data,
            self.ws.data_ptr(), self.ws.numel(), _stream(Xs[0]), ctypes.byref(self._plan)),
            "sng_batch_plan_create")

    def launch(self):
        check(_lib.load().sng_batch_plan_launch(self._plan, _stream(self.Xs[0])),
              "sng_batch_plan_launch")
        return self.labels, self.degrees

    def __del__(self):
        try:
            if self._plan:
                _lib.load().sng_batch_plan_destroy(self._plan)
                self._plan = None
        except Exception:
            pass
