"""Pins for the oracle's pair sampler (Algorithm 1, sampling step).

The sampler is Philox4x32-10 (Salmon et al., SC'11). Both word widths come
from one round macro in the oracle; the 64-bit instance is checked against
numpy's independent Philox4x64-10 and the 32-bit instance (and the sampler's
counter/key/word layout) against rocRAND's philox4x32_10 engine, compiled for
the host from its public headers.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox4x64_matches_numpy(orc):
    rng = np.random.default_rng(7)
    for _ in range(40):
        key = rng.integers(0, 2**64, size=2, dtype=np.uint64)
        ctr = rng.integers(0, 2**64, size=4, dtype=np.uint64)
        ctr[0] = ctr[0] % (2**63)  # no carry out of word 0 below
        bg = np.random.Philox(key=key, counter=ctr)
        raw = bg.random_raw(8)
        # numpy advances its counter before each block of four outputs
        c1 = ctr.copy(); c1[0] += np.uint64(1)
        c2 = ctr.copy(); c2[0] += np.uint64(2)
        assert np.array_equal(orc.philox4x64_10(c1, key), raw[:4])
        assert np.array_equal(orc.philox4x64_10(c2, key), raw[4:])


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rr_probe")
    subprocess.run([hipcc, "-O1", "--offload-host-only", "-o", exe,
                    os.path.join(HERE, "rocrand_philox_ref.hip")], check=True,
                   capture_output=True)
    return exe


def _rocrand(exe, triples):
    inp = "".join("%d %d %d\n" % t for t in triples)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64)


def test_philox4x32_matches_rocrand(orc, rocrand_probe):
    rng = np.random.default_rng(11)
    triples = [(0, 0, 0), (1, 0, 0), (2**64 - 1, 2**31 - 1, 2**32 - 1), (2**32, 1, 2**31)]
    for _ in range(200):
        triples.append((int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2)),
                        int(rng.integers(0, 2**31)), int(rng.integers(0, 2**32))))
    ref = _rocrand(rocrand_probe, triples)
    for (seed, i, c), r in zip(triples, ref):
        got = orc.philox4x32_10([c, i, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
        assert np.array_equal(got.astype(np.uint64), r), (seed, i, c)


def test_partner_layout_matches_rocrand(orc, rocrand_probe):
    """j = word (t mod 4) of Philox(ctr=(t/4, i, 0, 0), key=seed) mod n."""
    rng = np.random.default_rng(12)
    cases = []
    for _ in range(300):
        n = int(rng.choice([1, 2, 3, 7, 1000, 10**6, 5 * 10**6, 2**31 - 1]))
        cases.append((int(rng.integers(0, 2**64, dtype=np.uint64)), n,
                      int(rng.integers(0, n)), int(rng.integers(0, 2**34))))
    ref = _rocrand(rocrand_probe, [(s, i, t // 4) for s, n, i, t in cases])
    for (seed, n, i, t), r in zip(cases, ref):
        assert orc.partner(seed, n, i, t) == int(r[t % 4]) % n


def test_samples_per_point_closed_form(orc):
    # m = ceil(s*n) for the five workload shapes and the edges of the domain
    assert orc.samples_per_point(0.01, 10_000) == 100
    assert orc.samples_per_point(0.001, 1_000_000) == 1000
    assert orc.samples_per_point(0.01, 70_000) == 700
    assert orc.samples_per_point(0.002, 500_000) == 1000
    assert orc.samples_per_point(0.0005, 5_000_000) == 2500
    assert orc.samples_per_point(0.0, 123) == 0
    assert orc.samples_per_point(1.0, 123) == 123
    assert orc.samples_per_point(0.5, 3) == 2
    assert orc.samples_per_point(1e-9, 10) == 1
    assert orc.samples_per_point(-0.1, 10) == -1
    assert orc.samples_per_point(float("nan"), 10) == -1
    assert orc.samples_per_point(float("inf"), 10) == -1


def test_sampler_is_uniform(orc):
    """Partners are uniform on [0,n): chi-square over n cells, self rate ~1/n,
    and consecutive samples of a point are independent (chi-square on a 2-d
    grid of coarse cells)."""
    from scipy import stats
    n, m, seed = 257, 400, 99
    js = np.array([[orc.partner(seed, n, i, t) for t in range(m)] for i in range(n)])
    counts = np.bincount(js.ravel(), minlength=n)
    chi2 = ((counts - m) ** 2 / m).sum()
    assert stats.chi2.sf(chi2, n - 1) > 1e-4
    self_rate = (js == np.arange(n)[:, None]).mean()
    assert abs(self_rate - 1.0 / n) < 5 * np.sqrt((1.0 / n) / (n * m))
    a, b = js[:, :-1].ravel() * 8 // n, js[:, 1:].ravel() * 8 // n
    tab = np.zeros((8, 8))
    np.add.at(tab, (a, b), 1)
    cell = np.bincount(np.arange(n) * 8 // n, minlength=8) / n
    exp = tab.sum() * np.outer(cell, cell)
    assert stats.chi2.sf(((tab - exp) ** 2 / exp).sum(), 63) > 1e-4
