"""CPU tests of libg3's host side: the library loads, exports every entry
point that include/g3.h declares, validates arguments, and its exact
thresholds and ideal-gas normalisation agree with the (independent) oracle.
No compute call touches a GPU here."""
from __future__ import annotations

import math
import os
import re

import numpy as np
import pytest

from paper_1708_08619_amd import g3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "g3.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(g3.LIB_PATH):
        from paper_1708_08619_amd import build
        build.build()
    return g3.lib()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(g3_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s


def test_hist_len():
    assert g3.hist_len(60, g3.HALF) == 60 * 61 // 2 * 60 == 109800
    assert g3.hist_len(50, g3.FULL) == 125000
    assert g3.hist_len(0, 0) == 0 and g3.hist_len(g3.MAX_NBINS + 1, 0) == 0
    assert g3.hist_len(10, 7) == 0


@pytest.mark.parametrize("args,status", [
    ((256, [28016] * 3, 10240.0, 50, 1), g3.OK),
    ((65536, [174356] * 3, 12288.0, 60, 0), g3.OK),
    ((4096, [325600] * 3, 0.6 * 65536, 60, 1), g3.OK),
    ((256, [20000] * 3, 10240.0, 50, 1), g3.EINVAL),     # rmax >= L/2
    ((256, [28016] * 3, 0.5, 50, 1), g3.EINVAL),         # rmax < 1 unit
    ((256, [28016] * 3, 46341.0, 50, 1), g3.EINVAL),     # beyond the uint32 bound
    ((256, [28016] * 3, 10240.0, 0, 1), g3.EINVAL),
    ((256, [28016] * 3, 10240.0, g3.MAX_NBINS + 1, 1), g3.EINVAL),
    ((256, [28016] * 3, 10240.0, 50, 2), g3.EINVAL),     # layout
    ((-1, [28016] * 3, 10240.0, 50, 1), g3.EINVAL),
    ((256, [28016, 0, 28016], 10240.0, 50, 1), g3.EINVAL),
    ((256, [1 << 30] * 3, 10240.0, 50, 1), g3.EINVAL),   # box beyond 2^29
    ((256, [28016] * 3, float("nan"), 50, 1), g3.EINVAL),
])
def test_check_args(args, status):
    assert g3.check_args(*args) == status


@pytest.mark.parametrize("rmax,nbins", [
    (1000.0, 10), (10240.0, 50), (12288.0, 60), (0.6 * 65536, 60), (8192.0, 40),
    (123.456, 7), (46339.999, 160), (1.0, 1), (float.fromhex("0x1.3333333333333p+13"), 37),
])
def test_thresholds_match_oracle(oracle_mod, rmax, nbins):
    got = g3.thresholds(rmax, nbins).astype(np.uint64)
    assert np.array_equal(got, oracle_mod.thresholds(rmax, nbins))


def test_thresholds_random_match_oracle(oracle_mod):
    rng = np.random.default_rng(3)
    for _ in range(200):
        rmax = float(rng.uniform(1.0, 46340.0))
        nbins = int(rng.integers(1, g3.MAX_NBINS + 1))
        assert np.array_equal(g3.thresholds(rmax, nbins).astype(np.uint64),
                              oracle_mod.thresholds(rmax, nbins)), (rmax, nbins)


def test_ideal_volume_vs_oracle_and_closed_forms(oracle_mod):
    for nb, R in [(12, 1.0), (50, 10240.0), (7, 3.0)]:
        dr = R / nb
        W = g3.ideal_volume(nb, R)
        Wo = oracle_mod.W_table(nb, dr)
        scale = W.max()
        assert np.allclose(W, Wo, rtol=1e-12, atol=1e-13 * scale)
        assert math.isclose(W.sum(), (4 * math.pi / 3 * R ** 3) ** 2 * 15 / 32, rel_tol=1e-12)


@pytest.mark.parametrize("layout", [g3.HALF, g3.FULL])
def test_normalize_vs_oracle(oracle_mod, layout):
    nb, rmax, F, N, box = 20, 10240.0, 7, 256, [28016] * 3
    rng = np.random.default_rng(8 + layout)
    H = rng.integers(0, 1 << 40, size=g3.hist_len(nb, layout), dtype=np.uint64)
    got = g3.normalize(H, layout, nb, rmax, F, N, box)
    want = oracle_mod.normalize(H, layout, nb, rmax, F, N, box)
    live = want != 0
    assert np.array_equal(got == 0, want == 0)
    assert np.max(np.abs(got[live] / want[live] - 1.0)) < 1e-12


def test_normalize_rejects_bad_length():
    with pytest.raises(ValueError):
        g3.normalize(np.zeros(10, dtype=np.uint64), g3.HALF, 5, 100.0, 1, 10, [1000] * 3)


def test_normalize_pairs_vs_oracle(oracle_mod):
    nb, rmax, F, N, box = 60, 12288.0, 5, 65536, [174356] * 3
    rng = np.random.default_rng(21)
    H2 = rng.integers(0, 1 << 40, size=nb, dtype=np.uint64)
    got = g3.normalize_pairs(H2, nb, rmax, F, N, box)
    want = oracle_mod.normalize_pairs(H2, nb, rmax, F, N, box)
    assert np.max(np.abs(got / want - 1.0)) < 1e-12
    with pytest.raises(ValueError):
        g3.normalize_pairs(H2[:10], nb, rmax, F, N, box)


@pytest.mark.parametrize("layout", [g3.HALF, g3.FULL])
def test_superposition_vs_oracle(oracle_mod, layout):
    nb = 9
    rng = np.random.default_rng(30 + layout)
    full = rng.uniform(0.0, 3.0, (nb, nb, nb))
    full = (full + full.transpose(1, 0, 2)) / 2           # symmetric in the two centre sides
    g2 = rng.uniform(0.2, 2.0, nb)
    g2[4] = 0.0
    want = oracle_mod.superposition_full(full, g2)
    if layout == g3.FULL:
        src, want_l = full.reshape(-1), want.reshape(-1)
    else:
        idx = [(a, b, c) for a in range(nb) for b in range(a, nb) for c in range(nb)]
        src = np.array([full[i] for i in idx])
        want_l = np.array([want[i] for i in idx])
    got = g3.superposition(src, layout, nb, g2)
    assert np.allclose(got, want_l, rtol=1e-13, atol=0)


@pytest.mark.parametrize("layout", [g3.HALF, g3.FULL])
def test_isosceles_vs_oracle(oracle_mod, layout):
    nb = 12
    full = np.arange(nb ** 3, dtype=np.float64).reshape(nb, nb, nb)
    full = np.minimum(full, full.transpose(1, 0, 2))       # symmetric, distinct per (lo, hi, c)
    src = full.reshape(-1) if layout == g3.FULL else np.array(
        [full[a, b, c] for a in range(nb) for b in range(a, nb) for c in range(nb)])
    for a in (0, 3, 11):
        th, val = g3.isosceles(src, layout, nb, a)
        assert np.array_equal(val, full[a, a, :])
        want = np.array([oracle_mod.isosceles_angle(a, c) for c in range(nb)])
        assert np.allclose(th, want, rtol=1e-12, atol=1e-12)
    with pytest.raises(g3.G3Error):
        g3.isosceles(src, layout, nb, nb)
