"""The C ABI library loads on the CPU, exports every symbol include/sng.h
declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2006_06743_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2006_06743_amd import build
        build.build()
    return _lib.load()


def header_symbols():
    src = open(os.path.join(ROOT, "include", "sng.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sng_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lib):
    from paper_2006_06743_amd import _lib
    syms = header_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(_lib.EXPORTS) == syms


def test_status_strings(lib):
    for code in range(-6, 1):
        assert lib.sng_status_string(code)
    assert lib.sng_status_string(12345) == b"unknown status"


def test_samples_per_point(lib):
    m = ctypes.c_int64()
    for s, n, want in [(0.01, 10000, 100), (0.001, 10**6, 1000), (0.01, 70000, 700),
                       (0.002, 500000, 1000), (0.0005, 5 * 10**6, 2500), (0.0, 5, 0),
                       (1.0, 7, 7), (0.5, 3, 2)]:
        assert lib.sng_samples_per_point(s, n, ctypes.byref(m)) == 0
        assert m.value == want
    assert lib.sng_samples_per_point(-1.0, 5, ctypes.byref(m)) == -1
    assert lib.sng_samples_per_point(float("nan"), 5, ctypes.byref(m)) == -1
    assert lib.sng_samples_per_point(float("inf"), 5, ctypes.byref(m)) == -1
    assert lib.sng_samples_per_point(3.0, 2**31 - 1, ctypes.byref(m)) == -2


def test_workspace_sizes(lib):
    b = ctypes.c_size_t()
    assert lib.sng_workspace_size(10**6, 16, 1000, 0, ctypes.byref(b)) == 0
    big = b.value
    assert big >= 10**6 * 5 + 10**6 * 250 // 8
    assert lib.sng_workspace_size(10**5, 16, 1000, 0, ctypes.byref(b)) == 0
    assert b.value < big
    assert lib.sng_workspace_size(-1, 16, 10, 0, ctypes.byref(b)) == -1
    assert lib.sng_workspace_size(10, 0, 10, 0, ctypes.byref(b)) == -1
    assert lib.sng_workspace_size(10, 2, 10, 7, ctypes.byref(b)) == -1
    assert lib.sng_workspace_size(2**31, 2, 10, 0, ctypes.byref(b)) == -2


def test_invalid_arguments_rejected_before_launch(lib):
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    ws = ctypes.c_void_p(0x2000)
    lab = ctypes.c_void_p(0x3000)
    call = lambda **kw: lib.sng_dbscan(kw.get("X", fake), kw.get("n", 10), kw.get("d", 2),
                                       kw.get("ld", 2), kw.get("s", 0.5), kw.get("eps", 1.0),
                                       3, 1, kw.get("labels", lab), None, kw.get("ws", ws),
                                       kw.get("wsb", 0), None, None)
    assert call(d=0) == -1
    assert call(ld=1) == -1
    assert call(n=-1) == -1
    assert call(n=2**31) == -2
    assert call(eps=-0.5) == -1
    assert call(eps=float("nan")) == -1
    assert call(eps=float("inf")) == -1
    assert call(s=-0.1) == -1
    assert call(s=float("inf")) == -1
    assert call(s=2**40) == -2
    assert call(X=None) == -1
    assert call(X=ctypes.c_void_p(0x1002)) == -1  # not 4-byte aligned
    assert call(labels=None) == -1
    assert call(wsb=10) == -3          # workspace too small
    assert call(ws=None, wsb=10**9) == -3
    from paper_2006_06743_amd._lib import sng_config
    bad = sng_config(3, 0, 0, 0)
    assert lib.sng_dbscan(fake, 10, 2, 2, 0.5, 1.0, 3, 1, lab, None, ws, 10**9,
                          ctypes.byref(bad), None) == -1
    assert lib.sng_graph_labels(-1, None, 0, 1, lab, None, ws, 10**9, None) == -1
    assert lib.sng_graph_labels(5, None, 3, 1, lab, None, ws, 10**9, None) == -1
    assert lib.sng_graph_labels(5, fake, 3, 1, lab, None, ws, 1, None) == -3
    # compaction: null pointers, negative n, overlapping output, oversize n
    a = ctypes.c_void_p(0x10000)
    assert lib.sng_compact_labels(None, 5, a, None, None) == -1
    assert lib.sng_compact_labels(a, 5, None, None, None) == -1
    assert lib.sng_compact_labels(a, -1, a, None, None) == -1
    assert lib.sng_compact_labels(a, 5, ctypes.c_void_p(0x10000 + 16), None, None) == -1
    assert lib.sng_compact_labels(a, 2**31, ctypes.c_void_p(0x10000 + 2**33), None, None) == -2
    # sng_sample and the reuse_sample flag
    assert lib.sng_sample(-1, 2, 10, 1, ws, 10**9, None) == -1
    assert lib.sng_sample(10, 0, 10, 1, ws, 10**9, None) == -1
    assert lib.sng_sample(10, 2, -1, 1, ws, 10**9, None) == -1
    assert lib.sng_sample(10, 2, 2**31 + 1, 1, ws, 10**9, None) == -2
    assert lib.sng_sample(10, 2, 10, 1, ws, 10, None) == -3
    assert lib.sng_sample(10, 2, 10, 1, None, 10**9, None) == -3
    for fields in [(0, 0, 0, 0, 0, 2), (0, 0, 0, 0, 1, 1), (0, 0, 1, 0, 0, 1), (0, 0, 0, 0, 0, 0, 2)]:
        c = sng_config(*fields)
        assert lib.sng_dbscan(fake, 10, 2, 2, 0.5, 1.0, 3, 1, lab, None, ws, 10**9,
                              ctypes.byref(c), None) == -1, fields


def test_autotune_arguments_and_cache(lib):
    from paper_2006_06743_amd._lib import sng_config
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x2000)
    best = sng_config()
    ms = ctypes.c_float()
    # validation before any launch
    assert lib.sng_autotune(fake, 10, 2, 2, 5, 0.1, 1, ws, 10**9, 0, ctypes.byref(best),
                            None, None, None) == -1          # trials < 1
    assert lib.sng_autotune(fake, 10, 2, 2, 5, 0.1, 1, ws, 10**9, 2, None, None, None,
                            None) == -1                      # no output
    assert lib.sng_autotune(fake, 10, 2, 2, 5, -1.0, 1, ws, 10**9, 2, ctypes.byref(best),
                            None, None, None) == -1          # eps < 0
    assert lib.sng_autotune(fake, 10, 2, 2, 5, 0.1, 1, ws, 10, 2, ctypes.byref(best),
                            None, None, None) == -3          # workspace too small
    # nothing to tune: m = 0 returns an all-zero config without touching the device
    assert lib.sng_autotune(fake, 10, 2, 2, 0, 0.1, 1, ws, 10**9, 2, ctypes.byref(best),
                            ctypes.byref(ms), None, None) == 0
    assert best.schedule == 0 and best.lanes_per_pair == 0 and ms.value == 0.0
    assert lib.sng_autotune_clear() == 0
    out = sng_config()
    assert lib.sng_autotune_lookup(fake, 10, 2, 2, 5, ctypes.byref(out)) == -6
    assert lib.sng_autotune_lookup(fake, 10, 2, 2, 5, None) == -1


def test_similarity_arguments_rejected_before_launch(lib):
    from paper_2006_06743_amd._lib import sng_config
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x2000)
    lab = ctypes.c_void_p(0x3000)

    def call(**kw):
        return lib.sng_dbscan_similarity(kw.get("X", fake), kw.get("n", 10), kw.get("d", 2),
                                         kw.get("ld", 2), kw.get("s", 0.5), kw.get("kind", 2),
                                         kw.get("tau", 0.5), 3, 1, kw.get("labels", lab), None,
                                         kw.get("ws", ws), kw.get("wsb", 0), kw.get("cfg"), None)
    assert call(kind=0) == -1 and call(kind=3) == -1
    assert call(tau=float("nan")) == -1
    assert call(tau=float("inf")) == -1 and call(tau=float("-inf")) == -1
    assert call(d=0) == -1 and call(ld=1) == -1 and call(n=2**31) == -2
    assert call(s=-1.0) == -1 and call(labels=None) == -1
    assert call(wsb=10) == -3
    assert call(cfg=ctypes.byref(sng_config(0, 0, 0, 0, 0, 1))) == -1  # reuse_sample
    # workspace: the dot product adds nothing, the cosine a unit copy of the
    # rows (d rounded up to a multiple of 4)
    b, c = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.sng_workspace_size(1000, 18, 50, 0x100, ctypes.byref(c)) == 0
    assert lib.sng_similarity_workspace_size(1000, 18, 50, 1, 0x100, ctypes.byref(b)) == 0
    assert b.value == c.value
    assert lib.sng_similarity_workspace_size(1000, 18, 50, 2, 0x100, ctypes.byref(b)) == 0
    assert c.value + 4 * 1000 * 20 <= b.value <= c.value + 4 * 1000 * 20 + 256
    assert lib.sng_similarity_workspace_size(1000, 16, 50, 1, 1, ctypes.byref(b)) == -1
    assert lib.sng_similarity_workspace_size(1000, 16, 50, 0, 0, ctypes.byref(b)) == -1
    assert lib.sng_similarity_workspace_size(-1, 16, 50, 1, 0, ctypes.byref(b)) == -1
    assert lib.sng_similarity_workspace_size(2**31, 16, 50, 2, 0, ctypes.byref(b)) == -2


def test_simple_graph_config_and_workspace(lib):
    from paper_2006_06743_amd._lib import sng_config
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x2000)
    lab = ctypes.c_void_p(0x3000)
    for fields in [(0, 0, 0, 0, 0, 0, 0, 2), (0, 0, 0, 0, 0, 0, 1, 1), (0, 0, 0, 0, 2, 1, 0, 1)]:
        c = sng_config(*fields)
        assert lib.sng_dbscan(fake, 10, 2, 2, 0.5, 1.0, 3, 1, lab, None, ws, 10**9,
                              ctypes.byref(c), None) == -1, fields
    simple = sng_config(0, 0, 0, 0, 0, 0, 0, 1)
    # the mixed form and the sweep have no simple-graph mode
    assert lib.sng_dbscan_lowp(fake, 10, 2, 2, fake, 8, 1.0, 1, 0.5, 1.0, 3, 1, lab, None, ws,
                               10**9, ctypes.byref(simple), None) == -6
    e = (ctypes.c_double * 1)(1.0)
    mp = (ctypes.c_int32 * 1)(3)
    assert lib.sng_dbscan_sweep(fake, 10, 2, 2, 0.5, e, 1, mp, 1, 1, lab, None, ws, 10**9,
                                ctypes.byref(simple), None) == -6
    # the table: 8 bytes per entry, 2^ceil(log2(max(64, 2 n m))) entries
    b, c = ctypes.c_size_t(), ctypes.c_size_t()
    for n, m in [(10, 2), (1000, 50), (12345, 77)]:
        assert lib.sng_workspace_size(n, 3, m, 0x100, ctypes.byref(c)) == 0
        assert lib.sng_workspace_size(n, 3, m, 0x300, ctypes.byref(b)) == 0
        entries = 64
        while entries < 2 * n * m:
            entries *= 2
        assert b.value - c.value == 8 * entries
        assert lib.sng_similarity_workspace_size(n, 3, m, 1, 0x300, ctypes.byref(b)) == 0
        assert lib.sng_similarity_workspace_size(n, 3, m, 1, 0x100, ctypes.byref(c)) == 0
        assert b.value - c.value == 8 * entries
    assert lib.sng_workspace_size(100, 3, 5, 1 | 0x200, ctypes.byref(b)) == -1  # mixed form
    # the table is capped at 2^36 entries
    assert lib.sng_workspace_size(2**30, 3, 2**5, 0x300, ctypes.byref(b)) == 0  # 2nm = 2^36
    assert lib.sng_workspace_size(2**30, 3, 2**6, 0x300, ctypes.byref(b)) == -2
    assert lib.sng_similarity_workspace_size(2**30, 3, 2**6, 2, 0x200, ctypes.byref(b)) == -2
    assert lib.sng_dbscan(fake, 2**30, 3, 3, 2.0**-23, 1.0, 3, 1, lab, None, ws, 2**62,
                          ctypes.byref(simple), None) == -2
    # too small for the table
    assert lib.sng_workspace_size(1000, 3, 50, 0x100, ctypes.byref(c)) == 0
    assert lib.sng_dbscan(fake, 1000, 3, 3, 0.05, 1.0, 3, 1, lab, None, ws, c.value,
                          ctypes.byref(simple), None) == -3


def test_sweep_limits_as_documented(lib):
    """sng.h: 1 <= n_eps <= 64 finite, >= 0, strictly increasing eps;
    1 <= n_minpts <= 16; beyond the limits SNG_ERANGE, before any launch."""
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x2000)
    lab = ctypes.c_void_p(0x3000)
    b = ctypes.c_size_t()

    def sweep(eps, mps, wsb=0):
        e = (ctypes.c_double * max(1, len(eps)))(*eps)
        p = (ctypes.c_int32 * max(1, len(mps)))(*mps)
        return lib.sng_dbscan_sweep(fake, 10, 2, 2, 0.5, e, len(eps), p, len(mps), 1, lab, None,
                                    ws, wsb, None, None)

    grid = [0.1 * (k + 1) for k in range(64)]
    assert sweep(grid, [2] * 16) == -3            # limits met: only the workspace is short
    assert sweep(grid + [7.0], [2]) == -2         # 65 eps values
    assert sweep([0.1], [2] * 17) == -2           # 17 MinPts values
    assert sweep([], [2]) == -1 and sweep([0.1], []) == -1
    assert sweep([0.2, 0.1], [2]) == -1           # not increasing
    assert sweep([0.1, 0.1], [2]) == -1           # not strictly increasing
    assert sweep([-0.1, 0.1], [2]) == -1
    assert sweep([0.1, float("inf")], [2]) == -1
    assert sweep([0.0, 0.1], [-5, 2**31 - 1]) == -3
    assert lib.sng_sweep_workspace_size(10, 2, 5, 64, 16, ctypes.byref(b)) == 0
    assert lib.sng_sweep_workspace_size(10, 2, 5, 65, 16, ctypes.byref(b)) == -2
    assert lib.sng_sweep_workspace_size(10, 2, 5, 64, 17, ctypes.byref(b)) == -2


def test_config_round_trip_keeps_every_field():
    import paper_2006_06743_amd as sng
    from paper_2006_06743_amd._lib import sng_config
    c = sng_config(4, 8, 1, 16, 2, 1, 1, 1, 2, 16, 8192)
    back = sng._config_of(c)
    assert back == sng.Config(4, 8, 1, 16, 2, 1, 1, 1, 2, 16, 8192)
    assert ctypes.sizeof(sng_config) == 11 * 4


def test_noalloc_limits_before_any_device_work(lib):
    """sng_dbscan_noalloc refuses, before touching the device, a call whose
    workspace exceeds SNG_NOALLOC_SCRATCH_BYTES (32 MiB) and reuse_sample."""
    from paper_2006_06743_amd._lib import sng_config
    fake = ctypes.c_void_p(0x1000)
    lab = ctypes.c_void_p(0x3000)
    b = ctypes.c_size_t()
    assert lib.sng_workspace_size(10**6, 16, 1000, 0x100, ctypes.byref(b)) == 0
    assert b.value > 32 << 20
    assert lib.sng_dbscan_noalloc(fake, 10**6, 16, 16, 0.001, 2.0, 5, 2, lab, None, None,
                                  None) == -2
    assert lib.sng_dbscan_noalloc(fake, 10, 2, 2, -0.5, 1.0, 3, 1, lab, None, None, None) == -1
    assert lib.sng_dbscan_noalloc(fake, 10, 0, 2, 0.5, 1.0, 3, 1, lab, None, None, None) == -1
    reuse = sng_config(0, 0, 0, 0, 0, 1, 0, 0)
    assert lib.sng_dbscan_noalloc(fake, 10, 2, 2, 0.5, 1.0, 3, 1, lab, None,
                                  ctypes.byref(reuse), None) == -1


def test_tuned_shape_fields_are_validated(lib):
    """mfma_waves, mfma_ksteps and hook_blocks take the documented values
    only; a bad one is rejected before any device work."""
    from paper_2006_06743_amd._lib import sng_config
    fake = ctypes.c_void_p(0x1000)
    lab = ctypes.c_void_p(0x3000)
    for field, bad in [("mfma_waves", 3), ("mfma_waves", 8), ("mfma_ksteps", 2),
                       ("mfma_ksteps", 32), ("hook_blocks", 255), ("hook_blocks", 65537),
                       ("hook_blocks", -1)]:
        c = sng_config()
        setattr(c, field, bad)
        assert lib.sng_dbscan(fake, 10, 2, 2, 0.5, 0.1, 3, 1, lab, None, fake, 10**9,
                              ctypes.byref(c), None) == -1, (field, bad)


def test_tuners_reject_bad_arguments_before_launch(lib):
    from paper_2006_06743_amd._lib import sng_config
    fake = ctypes.c_void_p(0x1000)
    best = sng_config()
    # trials out of range, no output
    for trials, out in [(0, ctypes.byref(best)), (1001, ctypes.byref(best)), (2, None)]:
        assert lib.sng_autotune_lowp(fake, 10, 2, 2, fake, 8, 1.0, 1, 0.5, 0.1, 3, 1, fake, None,
                                     fake, 10**9, trials, out, None, None, None) == -1
        assert lib.sng_autotune_hook(fake, 10, 2, 2, 5, 0.1, 1, 3, fake, fake, fake, 10**9,
                                     trials, out, None, None, None) == -1
        assert lib.sng_autotune_batch(0, None, None, 2, None, None, None, None, None, None,
                                      None, fake, 10**9, trials, out, None, None, None) == -1
    # a precision the mixed form does not have
    assert lib.sng_autotune_lowp(fake, 10, 2, 2, fake, 8, 1.0, 0, 0.5, 0.1, 3, 1, fake, None,
                                 fake, 10**9, 2, ctypes.byref(best), None, None, None) == -1
    # an empty batch: nothing to tune, an all-zero config
    assert lib.sng_autotune_batch(0, None, None, 2, None, None, None, None, None, None, None,
                                  fake, 10**9, 2, ctypes.byref(best), None, None, None) == 0
    assert best.lanes_per_pair == 0 and best.prefetch == 0


def _entry(form, d, vec, lg_n, lg_m, fields):
    return " ".join(str(v) for v in [form, d, vec, lg_n, lg_m] + list(fields))


def test_autotune_cache_file_round_trip(lib, tmp_path):
    """A cache file loads into the cache (plain entries are found by lookup),
    saves back to the same text, and bad files change nothing."""
    from paper_2006_06743_amd._lib import sng_config
    fake = ctypes.c_void_p(0x1000)  # 16-byte aligned
    plain = _entry(0, 2, 1, 4, 3, [1, 8, 0, 8, 1, 0, 0, 0, 0, 0, 4096])
    bf16 = _entry(1, 784, 1, 17, 10, [0, 0, 0, 0, 0, 0, 0, 0, 2, 16, 0])
    batch = _entry(3, 3, 1, 18, 11, [1, 16, 0, 8, 0, 0, 0, 0, 0, 0, 0])
    good = tmp_path / "tune.txt"
    good.write_text("sng-autotune 1\n" + "\n".join([plain, bf16, batch]) + "\n")
    assert lib.sng_autotune_clear() == 0
    assert lib.sng_autotune_load(str(good).encode()) == 0
    out = sng_config()
    # n = 10 -> ceil(log2) 4, m = 5 -> 3, d = 2, ld = 4 (16-byte rows)
    assert lib.sng_autotune_lookup(fake, 10, 2, 4, 5, ctypes.byref(out)) == 0
    assert (out.lanes_per_pair, out.chunks_per_wave, out.prefetch, out.schedule,
            out.hook_blocks) == (1, 8, 8, 1, 4096)
    back = tmp_path / "back.txt"
    assert lib.sng_autotune_save(str(back).encode()) == 0
    assert back.read_text().splitlines() == ["sng-autotune 1", plain, bf16, batch]
    # bad files: nothing changes
    for text in ["sng-autotune 2\n" + plain + "\n",                         # version
                 "sng-autotune 1\n" + plain[:-5] + "\n",                     # short line
                 "sng-autotune 1\n" + plain + " 7\n",                        # trailing field
                 "sng-autotune 1\n" + _entry(0, 2, 1, 4, 3, [3] + [0] * 10) + "\n",  # lanes 3
                 "sng-autotune 1\n" + _entry(4, 2, 1, 4, 3, [0] * 11) + "\n",        # form 4
                 "sng-autotune 1\n" + _entry(0, 2, 1, 4, 3, [0] * 10 + [100]) + "\n"]:
        bad = tmp_path / "bad.txt"
        bad.write_text(text)
        assert lib.sng_autotune_clear() == 0
        assert lib.sng_autotune_load(str(bad).encode()) == -1, text
        assert lib.sng_autotune_lookup(fake, 10, 2, 4, 5, ctypes.byref(out)) == -6
    assert lib.sng_autotune_load(str(tmp_path / "missing.txt").encode()) == -7
    assert lib.sng_autotune_save(str(tmp_path / "no_dir" / "x.txt").encode()) == -7
    assert lib.sng_autotune_load(None) == -1 and lib.sng_autotune_save(None) == -1
    assert lib.sng_autotune_clear() == 0
