"""GPU parity of the mixed-precision form (sng_dbscan_lowp): the 16-bit copy
only filters; every undecided pair is re-decided in binary64, so degrees and
labels must equal the oracle's bit for bit."""
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


def lp_tensor(bits: np.ndarray, pad_to: int = 8):
    """uint16 [n, d] -> cuda int16 view [n, d] with row stride a multiple of 8."""
    import torch
    n, d = bits.shape
    ld = (d + pad_to - 1) // pad_to * pad_to
    buf = np.zeros((max(n, 1), ld), np.uint16)
    buf[:n, :d] = bits
    t = torch.from_numpy(buf.view(np.int16)).cuda()
    return t[:n, :d] if n > 0 else t[:0, :d]


def run_lowp(sng, X, bits, s, eps, min_pts, seed, prec, scale=1.0):
    import torch
    Xg = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    lab, deg, ws = sng.dbscan_lowp(Xg, lp_tensor(bits), s, eps, min_pts, seed, prec=prec,
                                   lp_scale=scale)
    torch.cuda.synchronize()
    st = sng.stats(ws)
    assert st.overflow == 0
    return lab.cpu().numpy(), deg.cpu().numpy().view(np.uint32), st


def assert_same(gl, gd, ref, what):
    bad = np.nonzero(gd != ref.deg)[0]
    assert bad.size == 0, "%s: %d degrees differ (first %s)" % (what, bad.size, bad[:5])
    bad = np.nonzero(gl != ref.labels)[0]
    assert bad.size == 0, "%s: %d labels differ (first %s)" % (what, bad.size, bad[:5])


def bits_for(X, prec, scale=1.0):
    Y = (X / np.float32(scale)).astype(np.float32)
    return wl.bf16_bits(Y) if prec == 1 else wl.fp16_bits(Y)


@pytest.fixture(scope="module")
def mnist_ref(orc):
    """The 70,000 x 784 workload and the oracle's result on it (computed once)."""
    W = wl.mnistlike_784d()
    return W, orc.dbscan(W.X, W.eps, W.min_pts, W.seed, s=W.s)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", [1, 2], ids=["bf16", "fp16"])
def test_mnistlike_784d_full(sng, mnist_ref, prec):
    W, ref = mnist_ref
    print("case", W.name, "prec", prec, flush=True)
    gl, gd, st = run_lowp(sng, W.X, bits_for(W.X, prec), W.s, W.eps, W.min_pts, W.seed, prec)
    assert_same(gl, gd, ref, "%s prec=%d" % (W.name, prec))
    assert st.accepted == ref.accepted and st.n_clusters == ref.n_clusters
    print("rechecked fraction %.5f" % (st.rechecked / st.slots), flush=True)
    assert 0 < st.rechecked < 0.05 * st.slots


@pytest.mark.timeout(600)
def test_mnistlike_784d_full_plain(sng, mnist_ref):
    """The plain binary32 path (the baseline the mixed form is timed against)
    on the same workload: identical to the oracle too."""
    import torch
    W, ref = mnist_ref
    Xg = torch.from_numpy(np.ascontiguousarray(W.X)).cuda()
    lab, deg, ws = sng.dbscan(Xg, W.s, W.eps, W.min_pts, W.seed)
    torch.cuda.synchronize()
    st = sng.stats(ws)
    assert_same(lab.cpu().numpy(), deg.cpu().numpy().view(np.uint32), ref, W.name + " plain")
    assert st.accepted == ref.accepted


def test_mnistlike_integer_copy(sng, orc):
    """8-bit images: the copy holds the integers 0..255 exactly (scale 1/255)."""
    W = wl.mnistlike_784d(n_per=1500)
    eps = 3.9
    q = W.meta["q"].astype(np.float32)
    bits = wl.bf16_bits(q)
    ref = orc.dbscan(W.X, eps, W.min_pts, W.seed, s=W.s)
    gl, gd, st = run_lowp(sng, W.X, bits, W.s, eps, W.min_pts, W.seed, 1, scale=1.0 / 255.0)
    assert_same(gl, gd, ref, "integer copy")
    assert st.rechecked < 0.002 * st.slots


CASES = []
_rng = np.random.default_rng(4242)
for _k in range(24):
    CASES.append((_k, int(_rng.choice([1, 2, 40, 200, 1500])),
                  int(_rng.choice([1, 3, 5, 16, 31, 32, 33, 64, 100, 257, 784, 1000])),
                  str(_rng.choice(["blobs", "grid", "uniform", "dupes"])),
                  float(_rng.choice([0.0, 0.01, 0.1, 0.5])), int(_rng.choice([1, 2]))))


@pytest.mark.parametrize("case", CASES, ids=["r%d_n%d_d%d_%s_s%g_p%d" % c for c in CASES])
def test_random_instances(sng, orc, case):
    k, n, d, kind, s, prec = case
    rng = np.random.default_rng(700 + k)
    X = wl.random_instance(rng, n, d, kind, spread=0.04)
    seed = int(rng.integers(0, 2**63))
    if n >= 2:
        smp = X[rng.integers(0, n, 50)].astype(np.float64)
        dd = np.sqrt(((smp[:, None] - smp[None]) ** 2).sum(-1))
        eps = float(np.quantile(dd[dd > 0], 0.2)) if np.any(dd > 0) else 1.0
    else:
        eps = 1.0
    print("case", case, "eps", eps, flush=True)
    for min_pts in [0, 2, 4]:
        ref = orc.dbscan(X, eps, min_pts, seed, s=s)
        gl, gd, _ = run_lowp(sng, X, bits_for(X, prec), s, eps, min_pts, seed, prec)
        assert_same(gl, gd, ref, "%s MinPts=%d" % (case, min_pts))


@pytest.mark.parametrize("prec", [1, 2], ids=["bf16", "fp16"])
def test_near_eps_adversarial(sng, orc, prec):
    """Points on a sphere of radius eps: almost every pair with the centre is
    undecided by the 16-bit filter and must come from the binary64 recheck."""
    rng = np.random.default_rng(31)
    for d in [3, 64, 300]:
        u = rng.normal(size=(2000, d))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        eps = 0.8
        X = np.vstack([np.zeros((300, d)), eps * u]).astype(np.float32)
        ref = orc.dbscan(X, eps, 3, 8, s=0.3)
        gl, gd, st = run_lowp(sng, X, bits_for(X, prec), 0.3, eps, 3, 8, prec)
        assert_same(gl, gd, ref, "sphere d=%d prec=%d" % (d, prec))
        assert st.rechecked > 0


def test_bad_copy_still_exact(sng, orc):
    """A copy that is far from X (wrong scale, NaNs) only costs rechecks."""
    rng = np.random.default_rng(5)
    X = wl.random_instance(rng, 800, 24, "blobs", spread=0.03)
    bits = wl.bf16_bits(X * 1.7)
    bits[::7, 3] = 0x7FC0  # NaN entries in the copy
    ref = orc.dbscan(X, 0.06, 3, 2, s=0.2)
    gl, gd, st = run_lowp(sng, X, bits, 0.2, 0.06, 3, 2, 1)
    assert_same(gl, gd, ref, "bad copy")


@pytest.mark.parametrize("prec", [1, 2], ids=["bf16", "fp16"])
def test_out_degree_mode_lowp(sng, orc, prec):
    """The mixed form with out-degrees equals the oracle's out-degree mode."""
    import torch
    rng = np.random.default_rng(77 + prec)
    X = wl.random_instance(rng, 3000, 48, "blobs", spread=0.05)
    seed = 31
    Xg = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    lab, deg, ws = sng.dbscan_lowp(Xg, lp_tensor(bits_for(X, prec)), 0.05, 0.4, 3, seed,
                                   prec=prec, cfg=sng.Config(out_degree=1))
    torch.cuda.synchronize()
    ref = orc.dbscan(X, 0.4, 3, seed, s=0.05, out_degree=True)
    assert_same(lab.cpu().numpy(), deg.cpu().numpy().view(np.uint32), ref, "lowp out-degree")


def _decode(bits, prec):
    b = np.ascontiguousarray(bits, dtype=np.uint16)
    if prec == 1:
        return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return b.view(np.float16).astype(np.float64)


@pytest.mark.parametrize("prec", [1, 2], ids=["bf16", "fp16"])
def test_filter_bound_is_reported_and_respected(sng, orc, prec):
    """The mixed form reports its filter: the accumulation bound, the rows'
    rounding radii r_i = ||x_i - scale v_i|| and the relative width at eps.
    On points at distance eps from a cluster centre, every slot whose copy
    distance T lies within r_i + r_j of eps must have been rechecked (then
    neither side of eps can be certain), and no slot outside the interval
    that the stated accumulation bound allows may have been."""
    import torch
    rng = np.random.default_rng(32 + prec)
    d, eps, s, seed, scale = 48, 0.8, 0.1, 8, 1.0
    u = rng.normal(size=(1200, d))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    X = np.vstack([rng.normal(0, 0.01, size=(200, d)), eps * u]).astype(np.float32)
    n = X.shape[0]
    bits = bits_for(X, prec, scale)
    Xg = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    lab, deg, ws = sng.dbscan_lowp(Xg, lp_tensor(bits), s, eps, 3, seed, prec=prec,
                                   lp_scale=scale)
    torch.cuda.synchronize()
    st = sng.stats(ws)
    ref = orc.dbscan(X, eps, 3, seed, s=s)
    assert_same(lab.cpu().numpy(), deg.cpu().numpy().view(np.uint32), ref, "sphere")
    # the stated constants, recomputed from the rows
    v = _decode(bits, prec)
    x = X.astype(np.float64)
    r = np.sqrt(((x - scale * v) ** 2).sum(1))
    a = np.sqrt((v ** 2).sum(1))
    u22 = 2.0 ** -22
    gamma = d * u22 / (1 - d * u22)
    gamma_norm = (2.0 * d + 24.0) * 2.0 ** -52
    assert st.filter_gamma == gamma
    assert r.max() * (1 - 1e-12) <= st.filter_r_max <= r.max() * (1 + 1e-9) + 1e-300
    assert abs(st.filter_r_mean - r.mean()) <= 1e-9 * r.mean() + 1e-300
    width = (2 * r.mean() + scale ** 2 * a.mean() ** 2 * (gamma + gamma_norm) / eps) / eps
    assert abs(st.filter_rel_width - width) <= 1e-6 * width
    assert st.band_rel == st.filter_rel_width
    # every slot: the copy's distance T and the interval the filter leaves open
    m = orc.samples_per_point(s, n)
    I = np.repeat(np.arange(n), m)
    J = np.array([orc.partner(seed, n, i, t) for i in range(n) for t in range(m)], np.int64)
    keep = I != J
    I, J = I[keep], J[keep]
    E = ((v[I] - v[J]) ** 2).sum(1)
    T = scale * np.sqrt(E)
    R = r[I] + r[J]
    delta = gamma * 2 * a[I] * a[J] + gamma_norm * (a[I] ** 2 + a[J] ** 2)
    t_lo = scale * np.sqrt(np.maximum(E - 2 * delta, 0.0))
    t_hi = scale * np.sqrt(E + 2 * delta)
    must = np.abs(T - eps) < R - 1e-9 * eps
    may = (t_lo - R <= eps * (1 + 1e-9)) & (t_hi + R >= eps * (1 - 1e-9))
    print("prec %d: must %d <= rechecked %d <= may %d of %d slots"
          % (prec, must.sum(), st.rechecked, may.sum(), I.size), flush=True)
    assert must.sum() > 0
    assert must.sum() <= st.rechecked <= may.sum()
    # the plain form reports no filter
    lab2, deg2, ws2 = sng.dbscan(Xg, s, eps, 3, seed)
    torch.cuda.synchronize()
    st2 = sng.stats(ws2)
    assert st2.filter_gamma == 0.0 and st2.filter_rel_width == 0.0


@pytest.mark.parametrize("prec", [1, 2], ids=["bf16", "fp16"])
def test_autotune_lowp_and_tuned_calls(sng, orc, prec, tmp_path):
    """The mixed form's tuner times waves per block x K-steps in flight
    (whole calls, each equal to the oracle), caches the fastest under its
    precision, and a call without a config then runs with it."""
    import torch
    W = wl.mnistlike_784d(n_per=300)
    X = W.X
    bits = bits_for(X, prec)
    s, eps = 0.05, 3.9
    ref = orc.dbscan(X, eps, W.min_pts, W.seed, s=s)
    Xg = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    sng.autotune_clear()
    print("autotune lowp", prec, flush=True)
    best, ms, tried, lab, deg = sng.autotune_lowp(Xg, lp_tensor(bits), s, eps, W.min_pts,
                                                  W.seed, prec=prec, trials=1)
    torch.cuda.synchronize()
    assert tried == 9 and ms > 0.0
    assert best.mfma_waves in (1, 2, 4) and best.mfma_ksteps in (4, 8, 16)
    assert_same(lab.cpu().numpy(), deg.cpu().numpy().view(np.uint32), ref, "last candidate")
    path = tmp_path / "tune.txt"
    sng.autotune_save(str(path))
    lines = path.read_text().splitlines()
    assert len(lines) == 2 and lines[1].startswith("%d 784 " % prec)
    gl, gd, _ = run_lowp(sng, X, bits, s, eps, W.min_pts, W.seed, prec)
    assert_same(gl, gd, ref, "tuned call")
    # every shape explicitly, against the oracle
    for w in (1, 2, 4):
        for k in (4, 8, 16):
            lab, deg, _ = sng.dbscan_lowp(Xg, lp_tensor(bits), s, eps, W.min_pts, W.seed,
                                          prec=prec, cfg=sng.Config(mfma_waves=w, mfma_ksteps=k))
            torch.cuda.synchronize()
            assert_same(lab.cpu().numpy(), deg.cpu().numpy().view(np.uint32), ref,
                        "waves %d ksteps %d" % (w, k))
    sng.autotune_clear()
