"""GPU parity of the batched forms: the hyperparameter sweep
(sng_dbscan_sweep) and many uneven instances (sng_dbscan_batch and its HIP
graph plan). Each result must equal the oracle's single run bit for bit."""
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


def assert_same(gl, gd, ref, what):
    bad = np.nonzero(gd != ref.deg)[0]
    assert bad.size == 0, "%s: %d degrees differ (first %s)" % (what, bad.size, bad[:5])
    bad = np.nonzero(gl != ref.labels)[0]
    assert bad.size == 0, "%s: %d labels differ (first %s)" % (what, bad.size, bad[:5])


SWEEP_CASES = [
    (0, 3000, 2, [0.01, 0.02, 0.03, 0.05], [1, 3, 6], 0.01),
    (1, 2500, 3, [0.02, 0.05, 0.1], [2, 4], 0.02),
    (2, 4000, 16, [0.05, 0.1, 0.15, 0.2, 0.3, 0.5, 0.8, 1.2], [0, 2, 4, 8], 0.01),
    (3, 1000, 33, [0.3], [3], 0.05),
    (4, 600, 5, np.linspace(0.01, 0.4, 20).tolist(), [-1, 1, 2, 3, 5, 8, 13], 0.1),
    (5, 1, 4, [0.1, 0.2], [0, 1], 1.0),
    (6, 2000, 8, [0.0, 0.05, 0.2], [1, 2], 0.0),
]


@pytest.mark.parametrize("schedule", [1, 2], ids=["direct", "partner_blocks"])
@pytest.mark.parametrize("case", SWEEP_CASES, ids=["s%d_n%d_d%d" % c[:3] for c in SWEEP_CASES])
def test_sweep_equals_single_runs(sng, orc, case, schedule):
    import torch
    k, n, d, eps, mps, s = case
    if schedule == 2 and d > 32:
        pytest.skip("partner-block schedule covers d <= 32")
    rng = np.random.default_rng(900 + k)
    X = wl.random_instance(rng, n, d, "blobs", spread=0.03)
    seed = int(rng.integers(0, 2**63))
    print("case", case[:3], "schedule", schedule, flush=True)
    labels, degs, ws = sng.sweep(gpu(X), s, eps, mps, seed, cfg=sng.Config(schedule=schedule))
    torch.cuda.synchronize()
    L = labels.cpu().numpy()
    D = degs.cpu().numpy().view(np.uint32)
    for ki, e in enumerate(eps):
        for pi, mp in enumerate(mps):
            ref = orc.dbscan(X, e, mp, seed, s=s)
            assert_same(L[pi, ki], D[ki], ref, "case %d eps=%g MinPts=%d" % (k, e, mp))


@pytest.fixture(scope="module")
def sweep_32d_reference(orc):
    """The oracle's 32 x 4 grid on the 500k x 32 workload: labels [4][32][n],
    degrees [32][n]."""
    W = wl.sweep_32d()
    labels, degs, _ = orc.sweep(W.X, W.eps_grid, W.min_pts_grid, W.seed, s=W.s)
    return W, labels, degs


@pytest.mark.timeout(600)
@pytest.mark.parametrize("schedule", [0, 1, 2], ids=["auto", "direct", "partner_blocks"])
def test_sweep_32d_full_size(sng, sweep_32d_reference, schedule):
    """The 500k x 32 workload with its 32 x 4 grid: all 32 degree rows and all
    128 label sets equal the oracle's single runs."""
    import torch
    W, ref_l, ref_d = sweep_32d_reference
    print("sweep 500k x 32, schedule", schedule, flush=True)
    labels, degs, ws = sng.sweep(gpu(W.X), W.s, W.eps_grid, W.min_pts_grid, W.seed,
                                 cfg=sng.Config(schedule=schedule))
    torch.cuda.synchronize()
    st = sng.stats(ws)
    L = labels.cpu().numpy()
    D = degs.cpu().numpy().view(np.uint32)
    assert st.accepted > 0
    for ki in range(len(W.eps_grid)):
        bad = np.nonzero(D[ki] != ref_d[ki])[0]
        assert bad.size == 0, "level %d: %d degrees differ (first %s)" % (ki, bad.size, bad[:5])
        for pi in range(len(W.min_pts_grid)):
            bad = np.nonzero(L[pi, ki] != ref_l[pi, ki])[0]
            assert bad.size == 0, "level %d MinPts %d: %d labels differ (first %s)" % (
                ki, W.min_pts_grid[pi], bad.size, bad[:5])
    # the grid spans all-noise to whole components
    assert (ref_l[0, 0] >= 0).mean() < 0.5 < (ref_l[0, -1] >= 0).mean()


def random_batch(rng, count, d=3):
    out = []
    for k in range(count):
        n = int(rng.choice([0, 1, 2, 17, 64, 65, 500, 3000, 20000]))
        out.append(wl.small_blobs_3d(n, 2000 + k, 300 + k) if d == 3 else None)
    return out


def check_batch(orc, B, labels, degs, what):
    for k, b in enumerate(B):
        ref = orc.dbscan(b.X, b.eps, b.min_pts, b.seed, s=b.s)
        assert_same(labels[k].cpu().numpy(), degs[k].cpu().numpy().view(np.uint32), ref,
                     "%s instance %d (n=%d)" % (what, k, b.n))


def test_batch_small_uneven(sng, orc):
    import torch
    rng = np.random.default_rng(17)
    B = random_batch(rng, 40)
    Xs = [gpu(b.X) for b in B]
    labels, degs, ws = sng.batch(Xs, [b.s for b in B], [b.eps for b in B],
                                 [b.min_pts for b in B], [b.seed for b in B])
    torch.cuda.synchronize()
    check_batch(orc, B, labels, degs, "direct")
    for k, b in enumerate(B):
        st = sng.stats(ws, k)
        assert st.slots == b.n * orc.samples_per_point(b.s, b.n)


def test_batch_plan_replays(sng, orc):
    """The captured graph replayed three times, with eager work on the same
    stream between replays; every replay must equal the oracle."""
    import torch
    rng = np.random.default_rng(23)
    B = random_batch(rng, 24)
    Xs = [gpu(b.X) for b in B]
    plan = sng.BatchPlan(Xs, [b.s for b in B], [b.eps for b in B], [b.min_pts for b in B],
                         [b.seed for b in B])
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(3):
        labels, degs = plan.launch()
        junk += 1.0  # eager work between replays
        torch.cuda.synchronize()
        check_batch(orc, B, labels, degs, "replay %d" % rep)
        for t in labels:
            t.fill_(-7)  # replays must rewrite every output
        for t in degs:
            t.fill_(12345)


@pytest.mark.timeout(600)
def test_batch_64_uneven_full(sng, orc):
    """The 64-instance workload (n log-uniform in [1e3, 2e5], d=3, s=0.01)."""
    import torch
    B = wl.uneven_batch()
    Xs = [gpu(b.X) for b in B]
    plan = sng.BatchPlan(Xs, [b.s for b in B], [b.eps for b in B], [b.min_pts for b in B],
                         [b.seed for b in B])
    labels, degs = plan.launch()
    torch.cuda.synchronize()
    check_batch(orc, B, labels, degs, "graph")


@pytest.mark.parametrize("schedule", [1, 2], ids=["direct", "partner_blocks"])
def test_sweep_out_degree(sng, orc, schedule):
    """The sweep with out-degrees equals single out-degree runs."""
    import torch
    rng = np.random.default_rng(4321)
    X = wl.random_instance(rng, 3000, 4, "blobs", spread=0.03)
    eps, mps, s, seed = [0.01, 0.03, 0.08], [1, 2, 4], 0.02, 99
    labels, degs, ws = sng.sweep(gpu(X), s, eps, mps, seed,
                                 cfg=sng.Config(schedule=schedule, out_degree=1))
    torch.cuda.synchronize()
    L = labels.cpu().numpy()
    D = degs.cpu().numpy().view(np.uint32)
    for ki, e in enumerate(eps):
        for pi, mp in enumerate(mps):
            ref = orc.dbscan(X, e, mp, seed, s=s, out_degree=True)
            assert_same(L[pi, ki], D[ki], ref, "eps=%g MinPts=%d" % (e, mp))


def test_autotune_batch_and_tuned_batches(sng, orc, tmp_path):
    """The batch tuner times its launch shapes on a batch (every candidate's
    results are the oracle's), caches the fastest under the batch's shape
    class, and batch() and BatchPlan then run with it."""
    import torch
    rng = np.random.default_rng(41)
    B = random_batch(rng, 20)
    Xs = [gpu(b.X) for b in B]
    args = ([b.s for b in B], [b.eps for b in B], [b.min_pts for b in B], [b.seed for b in B])
    sng.autotune_clear()
    print("autotune batch", flush=True)
    best, ms, tried, labels, degs = sng.autotune_batch(Xs, *args, trials=1)
    torch.cuda.synchronize()
    assert tried >= 2 and ms > 0.0 and best.lanes_per_pair >= 1
    check_batch(orc, B, labels, degs, "last candidate")
    path = tmp_path / "tune.txt"
    sng.autotune_save(str(path))
    lines = path.read_text().splitlines()
    assert lines[0] == "sng-autotune 1" and len(lines) == 2 and lines[1].startswith("3 ")
    labels, degs, _ = sng.batch(Xs, *args)
    torch.cuda.synchronize()
    check_batch(orc, B, labels, degs, "tuned batch")
    plan = sng.BatchPlan(Xs, *args)
    labels, degs = plan.launch()
    torch.cuda.synchronize()
    check_batch(orc, B, labels, degs, "tuned plan")
    sng.autotune_clear()
