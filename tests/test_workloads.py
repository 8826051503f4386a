"""Shapes of the seeded workloads, and the derived eps of the 784-d one."""
import json
import os

import numpy as np
import pytest

from paper_2006_06743_amd import workloads as w

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_shapes_and_determinism():
    W = w.blobs_2d()
    assert W.X.shape == (10000, 2) and W.X.dtype == np.float32 and W.X.flags.c_contiguous
    assert np.array_equal(W.X, w.blobs_2d().X)
    W = w.mixture_16d(n_total=20000)
    assert W.X.shape == (20000, 16)
    B = w.uneven_batch()
    ns = np.array([b.n for b in B])
    assert len(B) == 64 and ns.min() >= 1000 and ns.max() <= 200000


def test_bf16_rounding_is_rne():
    x = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-9, -2.5, 0.0, 65504.0], np.float32)
    b = w.bf16_to_f32(w.bf16_bits(x))
    assert b.tolist() == [1.0, 1.0, 1.0 + 2**-7, -2.5, 0.0, 65536.0]


def test_mnistlike_eps_matches_stored():
    stored = json.load(open(os.path.join(GOLD, "mnistlike_eps.json")))
    assert float(stored["eps"]) == w.MNISTLIKE_EPS
    assert float(stored["q_k"]) < w.MNISTLIKE_EPS ** 2 < float(stored["q_next"])


@pytest.mark.slow
def test_mnistlike_eps_rederived(orc):
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "derive", os.path.join(GOLD, "derive_mnistlike_eps.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    assert float(mod.derive()["eps"]) == w.MNISTLIKE_EPS


def test_balls_3d_geometry():
    """Three unit balls, equal weights, ceil(20 ln n) samples per point."""
    import math
    W, truth = w.balls_3d(30000)
    assert W.X.shape == (30000, 3) and W.X.dtype == np.float32
    assert W.meta["m"] == math.ceil(20 * math.log(30000))
    assert math.ceil(W.s * W.n) == W.meta["m"]
    centres = np.array([[0.0, 0.0, 0.0], [4.0, 0.0, 0.0], [2.0, 2.0 * math.sqrt(3.0), 0.0]])
    r = np.linalg.norm(W.X.astype(np.float64) - centres[truth], axis=1)
    assert r.max() <= 1.0 + 1e-6
    # uniform in the ball: P(r <= 1/2) = 1/8
    assert abs((r <= 0.5).mean() - 0.125) < 0.01
    counts = np.bincount(truth, minlength=3)
    assert np.all(np.abs(counts / 30000 - 1 / 3) < 0.02)
    # balls are more than 2 eps apart
    gaps = [np.linalg.norm(centres[a] - centres[b]) - 2 for a in range(3) for b in range(a)]
    assert min(gaps) > 2 * W.eps
