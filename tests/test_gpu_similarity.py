"""GPU parity of the similarity-threshold form (sng_dbscan_similarity:
dot product or cosine >= tau) against the CPU oracle: degrees and labels
identical bit for bit, on both schedules, every launch shape, exact ties,
zero / NaN / extreme-norm rows and the full-size workloads."""
import numpy as np
import pytest

from paper_2006_06743_amd import workloads as wl

pytestmark = pytest.mark.gpu

DOT, COS = 1, 2


@pytest.fixture(scope="module")
def sng():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2006_06743_amd as s
    s.load()
    return s


def to_gpu(X, pad=0, offset=0):
    import torch
    n, d = X.shape
    ld = d + pad
    buf = torch.zeros(offset + max(n, 1) * ld + 4, dtype=torch.float32, device="cuda:0")
    view = buf[offset:offset + n * ld].view(n, ld)[:, :d] if n > 0 else buf[:0].view(0, d)
    if n > 0:
        view.copy_(torch.from_numpy(X))
    return view


def run(sng, X, s, kind, tau, min_pts, seed, cfg=None, pad=0, offset=0):
    import torch
    Xg = to_gpu(X, pad, offset)
    labels, deg, ws = sng.dbscan_similarity(Xg, s, kind, tau, min_pts, seed, cfg=cfg)
    torch.cuda.synchronize()
    return labels.cpu().numpy(), deg.cpu().numpy().view(np.uint32), sng.stats(ws)


def check(sng, orc, X, s, kind, tau, min_pts, seed, what, **kw):
    gl, gd, st = run(sng, X, s, kind, tau, min_pts, seed, **kw)
    ref = orc.dbscan_similarity(X, kind, tau, min_pts, seed, s=s,
                                out_degree=bool(kw.get("cfg") and kw["cfg"].out_degree))
    bad = np.nonzero(gd != ref.deg)[0]
    assert bad.size == 0, "%s: %d degrees differ, first at %s" % (what, bad.size, bad[:5])
    bad = np.nonzero(gl != ref.labels)[0]
    assert bad.size == 0, "%s: %d labels differ, first at %s" % (what, bad.size, bad[:5])
    assert st.accepted == ref.accepted and st.self_pairs == ref.self_pairs
    assert st.n_core == ref.n_core and st.n_clusters == ref.n_clusters
    return ref, st


def quantile_tau(rng, X, kind, q):
    """A threshold at quantile q of the similarity of random pairs."""
    n = X.shape[0]
    a, b = rng.integers(0, n, 256), rng.integers(0, n, 256)
    A, B = X[a].astype(np.float64), X[b].astype(np.float64)
    v = (A * B).sum(1)
    if kind == COS:
        v = v / np.maximum(np.linalg.norm(A, axis=1) * np.linalg.norm(B, axis=1), 1e-300)
    return float(np.quantile(v, q))


CASES = []
_rng = np.random.default_rng(4242)
for _k in range(36):
    _n = int(_rng.choice([0, 1, 2, 63, 65, 257, 1000, 3001]))
    _d = int(_rng.choice([1, 2, 3, 4, 5, 8, 9, 16, 17, 33, 64, 100, 784]))
    _kind = int(_rng.choice([DOT, COS]))
    _data = str(_rng.choice(["blobs", "uniform", "dupes", "grid"]))
    _s = float(_rng.choice([0.003, 0.01, 0.05, 0.3, 1.0]))
    _pad = int(_rng.choice([0, 0, 1, 4]))
    CASES.append((_k, _n, _d, _kind, _data, _s, _pad))


@pytest.mark.parametrize("case", CASES, ids=["r%d_n%d_d%d_k%d_%s_s%g_p%d" % c for c in CASES])
def test_random_instances(sng, orc, case):
    k, n, d, kind, data, s, pad = case
    rng = np.random.default_rng(9000 + k)
    X = wl.random_instance(rng, n, d, data, spread=0.05)
    X = (X - 0.5).astype(np.float32)  # signs of both kinds, so dot products cancel
    seed = int(rng.integers(0, 2**64, dtype=np.uint64))
    tau = quantile_tau(rng, X, kind, rng.uniform(0.5, 0.98)) if n >= 2 else 0.1
    print("case", case, "tau", tau, flush=True)
    for min_pts in [0, 2, 5]:
        check(sng, orc, X, s, kind, tau, min_pts, seed, "%s MinPts=%d" % (case, min_pts),
              pad=pad)


@pytest.mark.parametrize("kind", [DOT, COS])
def test_exact_ties_with_the_definition(sng, orc, kind):
    """tau taken from the oracle's own value for sampled pairs: those pairs
    sit exactly on the threshold, where only the binary64 definition (its
    rounding of products, square roots and quotient) decides."""
    rng = np.random.default_rng(31 + kind)
    n, d, s, seed = 2000, 7, 0.01, 77
    X = rng.normal(size=(n, d)).astype(np.float32)
    m = orc.samples_per_point(s, n)
    f = orc.dot if kind == DOT else orc.cosine
    for trial in range(6):
        i = int(rng.integers(0, n))
        j = orc.partner(seed, n, i, int(rng.integers(0, m)))
        if j == i:
            continue
        tau = f(X, i, j)
        print("tie", kind, i, j, tau, flush=True)
        ref, st = check(sng, orc, X, s, kind, tau, 1, seed, "tie %d" % trial)
        assert st.rechecked >= 1


def test_integer_dot_ties(sng, orc):
    """Small integers: dot products are exact integers and many slots tie
    with an integer tau; every tie goes through the binary64 recheck."""
    rng = np.random.default_rng(5)
    X = rng.integers(-4, 5, size=(5000, 5)).astype(np.float32)
    for tau in [0.0, 3.0, 9.0, -2.0]:
        ref, st = check(sng, orc, X, 0.02, DOT, tau, 4, 11, "int tau=%g" % tau)
        assert st.rechecked > 0


def test_zero_nan_and_extreme_rows(sng, orc):
    """Zero rows (no cosine), NaN and infinite rows, and rows whose squared
    norm is outside [2^-100, 2^100] (decided in binary64 throughout)."""
    rng = np.random.default_rng(6)
    X = rng.normal(size=(3000, 6)).astype(np.float32)
    X[::7] = 0.0
    X[3::11, 2] = np.nan
    X[5::13, 0] = np.inf
    X[1::17] *= np.float32(2.0 ** -60)
    X[2::19] *= np.float32(2.0 ** 55)
    for kind, tau in [(COS, 0.5), (COS, -0.3), (DOT, 0.0), (DOT, -1.0), (DOT, 2.0)]:
        check(sng, orc, X, 0.05, kind, tau, 2, 3, "extreme kind=%d tau=%g" % (kind, tau))


@pytest.mark.parametrize("d", [3, 16, 100])
def test_every_launch_shape_is_identical(sng, orc, d):
    rng = np.random.default_rng(88 + d)
    X = (wl.random_instance(rng, 2500, d, "blobs", spread=0.02) - 0.5).astype(np.float32)
    for kind in [DOT, COS]:
        tau = quantile_tau(rng, X, kind, 0.9)
        ref = orc.dbscan_similarity(X, kind, tau, 3, 123, s=0.02)
        shapes = [(lanes, cpw, lds, pf, sc) for lanes in [0, 1, 4, 16, 64] for cpw in [1, 64]
                  for lds in [0, 1] for pf in [0, 8] for sc in ([0, 1, 2] if d <= 32 else [0, 1])
                  if not (lds and (pf or sc == 2))]
        for lanes, cpw, lds, pf, sc in shapes:
            cfg = sng.Config(lanes, cpw, lds, pf, sc)
            print("shape d=%d kind=%d cfg=%s" % (d, kind, cfg), flush=True)
            gl, gd, _ = run(sng, X, 0.02, kind, tau, 3, 123, cfg=cfg)
            assert np.array_equal(gd, ref.deg) and np.array_equal(gl, ref.labels), cfg


@pytest.mark.parametrize("kind", [DOT, COS])
def test_out_degree_mode(sng, orc, kind):
    rng = np.random.default_rng(12 + kind)
    X = rng.normal(size=(4000, 8)).astype(np.float32)
    tau = quantile_tau(rng, X, kind, 0.8)
    for sc in [1, 2]:
        check(sng, orc, X, 0.02, kind, tau, 3, 8, "out-degree sc=%d" % sc,
              cfg=sng.Config(schedule=sc, out_degree=1))


def test_mixture_16d_full_size_cosine(sng, orc):
    """The 1e6 x 16 mixture (1e9 slots, partner-block schedule) with a cosine
    threshold: every label and degree against the whole oracle method."""
    W = wl.mixture_16d()
    print("case", W.name, "cosine 0.95", flush=True)
    ref, st = check(sng, orc, W.X, W.s, COS, 0.95, W.min_pts, W.seed, W.name)
    assert ref.n_core > 100000 and ref.n_clusters >= 50


def test_mnistlike_784d_cosine(sng, orc):
    """70k x 784 quantised images, 4.9e7 slots, cosine >= 0.9."""
    W = wl.mnistlike_784d()
    print("case", W.name, "cosine 0.9", flush=True)
    ref, st = check(sng, orc, W.X, W.s, COS, 0.9, 10, W.seed, W.name)
    assert ref.accepted > 0
