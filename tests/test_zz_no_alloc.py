"""sng_dbscan_noalloc (the allocation-free entry point, whose workspace is
the library's static device array) against sng_dbscan with a caller
workspace: identical labels and degrees on two calls in a row, the second
with a smaller input, through the C ABI."""
import ctypes

import numpy as np
import pytest

from paper_2006_06743_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2006_06743_amd import _lib
    return _lib.load()


def _with_workspace(lib, X, s, eps, mp, seed, cfg):
    import torch
    n, d = X.shape
    m = ctypes.c_int64()
    assert lib.sng_samples_per_point(s, n, ctypes.byref(m)) == 0
    b = ctypes.c_size_t()
    flags = 0x200 if (cfg is not None and cfg.simple_graph) else 0
    assert lib.sng_workspace_size(n, d, m.value, flags, ctypes.byref(b)) == 0
    ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device="cuda")
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    deg = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    rc = lib.sng_dbscan(X.data_ptr(), n, d, d, s, eps, mp, seed, lab.data_ptr(), deg.data_ptr(),
                        ws.data_ptr(), ws.numel(), ctypes.byref(cfg) if cfg else None, st)
    assert rc == 0
    return lab, deg


def _noalloc(lib, X, s, eps, mp, seed, cfg, with_degrees=True):
    import torch
    n, d = X.shape
    lab = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    deg = torch.full((n,), 12345, dtype=torch.int32, device="cuda") if with_degrees else None
    st = torch.cuda.current_stream().cuda_stream
    rc = lib.sng_dbscan_noalloc(X.data_ptr(), n, d, d, s, eps, mp, seed, lab.data_ptr(),
                                deg.data_ptr() if deg is not None else None,
                                ctypes.byref(cfg) if cfg else None, st)
    assert rc == 0, rc
    return lab, deg


CASES = [
    # (name, points, s, eps, MinPts, seed); the second case is the smaller
    ("blobs2d_n10k", lambda: wl.blobs_2d().X, 0.01, 0.05, 3, 1),
    ("blobs3d_n3000", lambda: wl.random_instance(np.random.default_rng(5), 3000, 3, "blobs",
                                                 spread=0.03), 0.02, 0.04, 2, 77),
]


@pytest.mark.parametrize("cfg_kind", ["default", "direct", "simple_graph"])
def test_noalloc_equals_workspace_call(lib, cfg_kind):
    import torch
    from paper_2006_06743_amd._lib import sng_config
    cfg = {"default": None, "direct": sng_config(0, 0, 0, 0, 1, 0, 0, 0),
           "simple_graph": sng_config(0, 0, 0, 0, 0, 0, 0, 1)}[cfg_kind]
    for name, make, s, eps, mp, seed in CASES:
        print("noalloc", cfg_kind, name, flush=True)
        X = torch.from_numpy(np.ascontiguousarray(make())).cuda()
        ref_l, ref_d = _with_workspace(lib, X, s, eps, mp, seed, cfg)
        got_l, got_d = _noalloc(lib, X, s, eps, mp, seed, cfg)
        torch.cuda.synchronize()
        assert torch.equal(got_d, ref_d), name
        assert torch.equal(got_l, ref_l), name
        assert int((ref_l >= 0).sum()) > 0, name  # some clusters form
    # degrees may be NULL; a repeat of the larger case after the smaller one
    name, make, s, eps, mp, seed = CASES[0]
    X = torch.from_numpy(np.ascontiguousarray(make())).cuda()
    ref_l, _ = _with_workspace(lib, X, s, eps, mp, seed, cfg)
    got_l, _ = _noalloc(lib, X, s, eps, mp, seed, cfg, with_degrees=False)
    torch.cuda.synchronize()
    assert torch.equal(got_l, ref_l)


def test_noalloc_rejects_oversize(lib):
    """A workload whose workspace exceeds the static array is refused
    before any work (1e6 points, 1000 samples each: about 130 MB)."""
    import torch
    X = torch.zeros((1_000_000, 16), dtype=torch.float32, device="cuda")
    lab = torch.empty(1_000_000, dtype=torch.int32, device="cuda")
    rc = lib.sng_dbscan_noalloc(X.data_ptr(), 1_000_000, 16, 16, 0.001, 2.0, 5, 2,
                                lab.data_ptr(), None, None, None)
    assert rc == -2
