"""GPU parity of the simple-graph degree mode (sng_config.simple_graph: a
point's degree counts its distinct accepted neighbours) against the oracle,
on both schedules, the distance and similarity queries, the degrees entry
point, heavy duplication (m close to n) and the full-size 1e6 x 16 mixture."""
import numpy as np
import pytest

from paper_2006_06743_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sng():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2006_06743_amd as s
    s.load()
    return s


def gpu(X):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X)).cuda()


def same(got_l, got_d, ref, what):
    got_d = got_d.cpu().numpy().view(np.uint32)
    got_l = got_l.cpu().numpy()
    bad = np.nonzero(got_d != ref.deg)[0]
    assert bad.size == 0, "%s: %d degrees differ, first at %s" % (what, bad.size, bad[:5])
    bad = np.nonzero(got_l != ref.labels)[0]
    assert bad.size == 0, "%s: %d labels differ, first at %s" % (what, bad.size, bad[:5])


CASES = [(0, 1, 2, 0.5), (1, 2, 2, 1.0), (2, 64, 3, 1.0), (3, 500, 2, 1.0), (4, 700, 5, 0.6),
         (5, 3001, 3, 0.05), (6, 2000, 16, 0.2), (7, 4000, 8, 0.01), (8, 1000, 33, 0.3)]


@pytest.mark.parametrize("case", CASES, ids=["c%d_n%d_d%d_s%g" % c for c in CASES])
@pytest.mark.parametrize("sched", [1, 2])
def test_distance_query(sng, orc, case, sched):
    import torch
    k, n, d, s = case
    rng = np.random.default_rng(700 + k)
    X = wl.random_instance(rng, n, d, "blobs", spread=0.05)
    eps = 0.15 * np.sqrt(d)
    seed = int(rng.integers(0, 2**63))
    print("case", case, "schedule", sched, flush=True)
    if sched == 2 and d > 32:
        sched = 0  # partner blocks cover d <= 32: let the library choose
    for mp in [0, 3, 20]:
        cfg = sng.Config(schedule=sched, simple_graph=1)
        lab, deg, ws = sng.dbscan(gpu(X), s, eps, mp, seed, cfg=cfg)
        torch.cuda.synchronize()
        ref = orc.dbscan(X, eps, mp, seed, s=s, simple_graph=True)
        same(lab, deg, ref, "%s MinPts=%d" % (case, mp))
        st = sng.stats(ws)
        assert st.accepted == ref.accepted and st.n_core == ref.n_core
        assert st.overflow == 0


@pytest.mark.parametrize("kind", [1, 2])
def test_similarity_queries(sng, orc, kind):
    import torch
    rng = np.random.default_rng(710 + kind)
    X = (wl.random_instance(rng, 3000, 6, "blobs", spread=0.05) - 0.5).astype(np.float32)
    tau = 0.9 if kind == 2 else 0.05
    for sched in [1, 2]:
        cfg = sng.Config(schedule=sched, simple_graph=1)
        lab, deg, _ = sng.dbscan_similarity(gpu(X), 0.1, kind, tau, 4, 5, cfg=cfg)
        torch.cuda.synchronize()
        ref = orc.dbscan_similarity(X, kind, tau, 4, 5, s=0.1, simple_graph=True)
        same(lab, deg, ref, "kind=%d schedule=%d" % (kind, sched))


def test_degrees_entry_point(sng, orc):
    import torch
    rng = np.random.default_rng(720)
    X = wl.random_instance(rng, 5000, 3, "blobs", spread=0.03)
    m = 300
    deg, _ = sng.degrees(gpu(X), m, 0.08, 9, cfg=sng.Config(simple_graph=1))
    torch.cuda.synchronize()
    ref = orc.dbscan(X, 0.08, 1, 9, m=m, simple_graph=True)
    assert np.array_equal(deg.cpu().numpy().view(np.uint32), ref.deg)


def test_reused_workspace_and_repeated_calls(sng, orc):
    """The table is cleared to the size each call needs: a dense call after a
    sparse one (and the reverse) in one workspace gives exact degrees."""
    import torch
    rng = np.random.default_rng(730)
    X = wl.random_instance(rng, 4000, 2, "blobs", spread=0.05)
    cfg = sng.Config(simple_graph=1)
    lab, deg, ws = sng.dbscan(gpu(X), 0.05, 0.5, 3, 1, cfg=cfg)
    for eps in [0.001, 0.5, 0.02, 1e30]:
        sng.dbscan(gpu(X), 0.05, eps, 3, 1, cfg=cfg, labels=lab, degrees_out=deg, ws=ws)
        torch.cuda.synchronize()
        same(lab, deg, orc.dbscan(X, eps, 3, 1, s=0.05, simple_graph=True), "eps=%g" % eps)


def test_mixture_16d_full_size(sng, orc):
    """The 1e6 x 16 mixture at sigma = 0.25 (dense), 1e9 slots, partner blocks."""
    import torch
    W = wl.mixture_16d(sigma=0.25)
    print("case", W.name, flush=True)
    lab, deg, ws = sng.dbscan(gpu(W.X), W.s, W.eps, W.min_pts, W.seed,
                              cfg=sng.Config(simple_graph=1))
    torch.cuda.synchronize()
    ref = orc.dbscan(W.X, W.eps, W.min_pts, W.seed, s=W.s, simple_graph=True)
    same(lab, deg, ref, W.name)
    assert ref.accepted > 10**6
