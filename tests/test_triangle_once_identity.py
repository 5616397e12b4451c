"""The triangle-once identity, checked on the CPU against the oracle.

Counting each triangle once, at its lowest-index atom, into T(lo, hi, c)
(lo <= hi the bins of the two sides at that atom, c the opposite side) and
then giving each output bin (x <= y, z) of the half histogram
    T(x,y,z) + [x<=z] T(x,z,y) + [x!=y][y<=z] T(y,z,x)
             + [z<=x] T(z,x,y) + [x!=y][z<=y] T(z,y,x)
reproduces the per-centre definition exactly whenever 2 rmax < L on every
axis: a side shorter than rmax < L/2 is its own minimum image, so the three
atoms of a counted triangle see the same three side vectors.  T here is a
brute-force count written for this test; the oracle is untouched."""
from __future__ import annotations

import numpy as np
import pytest

import refs


def _tri_counts(fr, box, rmax, nbins):
    F, _, N = fr.shape
    T = np.zeros((nbins, nbins, nbins), dtype=np.int64)
    for f in range(F):
        X = fr[f].astype(np.int64)
        for i in range(N):
            d = {}
            for j in range(i + 1, N):
                v = [refs.min_image(int(X[a, j] - X[a, i]), box[a]) for a in range(3)]
                b = refs.frac_bin(sum(x * x for x in v), rmax, nbins)
                if b >= 0:
                    d[j] = (v, b)
            js = sorted(d)
            for p, j in enumerate(js):
                for k in js[p + 1:]:
                    (vj, bj), (vk, bk) = d[j], d[k]
                    c = refs.frac_bin(sum((vk[a] - vj[a]) ** 2 for a in range(3)), rmax, nbins)
                    if c >= 0:
                        T[min(bj, bk), max(bj, bk), c] += 1
    return T


def _expand_half(T):
    nb = T.shape[0]
    out = []
    for x in range(nb):
        for y in range(x, nb):
            for z in range(nb):
                v = T[x, y, z]
                if x <= z:
                    v += T[x, z, y]
                if x != y and y <= z:
                    v += T[y, z, x]
                if z <= x:
                    v += T[z, x, y]
                if x != y and z <= y:
                    v += T[z, y, x]
                out.append(v)
    return np.array(out, dtype=np.uint64)


@pytest.mark.parametrize("seed", range(5))
def test_triangle_once_expands_to_the_definition(oracle_mod, seed):
    rng = np.random.default_rng(700 + seed)
    box = [int(x) for x in rng.integers(300, 700, size=3)]
    # rmax between L/3 and L/2 of the smallest side in some cases
    lo = min(box) / (2.6 if seed % 2 else 5.0)
    rmax = float(rng.uniform(lo, min(box) / 2 - 1))
    nbins = int(rng.integers(3, 8))
    N = int(rng.integers(8, 16))
    fr = np.stack([np.stack([rng.integers(0, L, size=N) for L in box]) for _ in range(2)]
                  ).astype(np.int32)
    got = _expand_half(_tri_counts(fr, box, rmax, nbins))
    want = oracle_mod.hist(fr, box, rmax, nbins, 0)
    assert want.sum() > 0
    assert np.array_equal(got, want)
