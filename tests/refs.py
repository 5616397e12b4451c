"""Independent reference computations used to pin the oracle.

None of these share code with ``oracle/`` or with the library:

* :func:`brute_full` -- O(F N^3) Python loops with thresholds decided in exact
  rational arithmetic (``fractions.Fraction`` of the binary64 rmax), i.e. the
  triplet definition of Sec. 3.3 written out with no neighbour lists.
* :func:`triangles_full` -- a different formulation of the same count: each
  triangle {i, j, k} (i < j < k) whose three minimum-image sides are shorter
  than rmax and *close* (d_ij + d_jk + d_ki = 0) is enumerated once and
  credited to all six ordered (centre, j, k) arrangements.
* :func:`lattice_full` -- perfect lattices: every site sees the same set of
  neighbour vectors (or its inversion), so H_full = N x (count over pairs of
  lattice vectors), computed from lattice vectors only.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def frac_bin_n(s: int, rmax: float, nbins: int, count: int) -> int:
    """Bins of width rmax / nbins, count of them: max{b : s >= (b rmax /
    nbins)^2} if s < (count rmax / nbins)^2, else -1 (exact)."""
    R = Fraction(rmax)
    lhs = Fraction(s) * nbins * nbins
    if lhs >= Fraction(count * count) * R * R:
        return -1
    b = 0
    while b + 1 < count and lhs >= Fraction((b + 1) ** 2) * R * R:
        b += 1
    return b


def frac_bin(s: int, rmax: float, nbins: int) -> int:
    """max{b : s >= (b rmax / nbins)^2} if s < rmax^2, else -1 (exact)."""
    R = Fraction(rmax)
    if Fraction(s) >= R * R:
        return -1
    # s * nbins^2 >= b^2 rmax^2
    lhs = Fraction(s) * nbins * nbins
    b = 0
    while b + 1 < nbins and lhs >= Fraction((b + 1) ** 2) * R * R:
        b += 1
    return b


def min_image(d: int, L: int) -> int:
    if 2 * d > L:
        return d - L
    if 2 * d < -L:
        return d + L
    return d


def brute_full(frames, box, rmax: float, nbins: int, nbins_third: int | None = None) -> np.ndarray:
    nc = nbins_third or nbins
    fr = np.asarray(frames, dtype=np.int64)
    F, _, N = fr.shape
    H = np.zeros((nbins, nbins, nc), dtype=np.uint64)
    cache: dict[int, int] = {}
    cache3: dict[int, int] = {}

    def b(s):
        if s not in cache:
            cache[s] = frac_bin(s, rmax, nbins)
        return cache[s]

    def b3(s):
        if s not in cache3:
            cache3[s] = frac_bin_n(s, rmax, nbins, nc)
        return cache3[s]

    for f in range(F):
        P = [tuple(int(fr[f, d, a]) for d in range(3)) for a in range(N)]
        for i in range(N):
            for j in range(N):
                if j == i:
                    continue
                dij = [min_image(P[j][d] - P[i][d], box[d]) for d in range(3)]
                bij = b(sum(x * x for x in dij))
                if bij < 0:
                    continue
                for k in range(N):
                    if k == i or k == j:
                        continue
                    dik = [min_image(P[k][d] - P[i][d], box[d]) for d in range(3)]
                    bik = b(sum(x * x for x in dik))
                    if bik < 0:
                        continue
                    djk = [dik[d] - dij[d] for d in range(3)]   # updated positions
                    bjk = b3(sum(x * x for x in djk))
                    if bjk < 0:
                        continue
                    H[bij, bik, bjk] += 1
    return H


def _bins_np(s: np.ndarray, rmax: float, nbins: int, count: int | None = None) -> np.ndarray:
    """Exact bins for an int64 array via per-value Fraction decisions."""
    out = np.empty(s.shape, dtype=np.int64)
    flat = s.reshape(-1)
    o = out.reshape(-1)
    uniq, inv = np.unique(flat, return_inverse=True)
    ub = np.array([frac_bin_n(int(v), rmax, nbins, count or nbins) for v in uniq], dtype=np.int64)
    o[:] = ub[inv]
    return out


def triangles_full(frames, box, rmax: float, nbins: int) -> np.ndarray:
    """H_full from closed triangles, each enumerated once (i < j < k)."""
    fr = np.asarray(frames, dtype=np.int64)
    F, _, N = fr.shape
    box = np.asarray(box, dtype=np.int64)
    H = np.zeros((nbins, nbins, nbins), dtype=np.uint64)
    for f in range(F):
        X = fr[f].T                                      # [N, 3]
        D = X[None, :, :] - X[:, None, :]                # D[i, j] = x_j - x_i
        D = np.where(2 * D > box, D - box, D)
        D = np.where(2 * D < -box, D + box, D)
        S = (D * D).sum(-1)
        B = _bins_np(S, rmax, nbins)                     # -1 where cut
        for i in range(N):
            js = np.nonzero((B[i] >= 0) & (np.arange(N) > i))[0]
            if len(js) < 2:
                continue
            jj, kk = np.meshgrid(js, js, indexing="ij")
            m = kk > jj
            jj, kk = jj[m], kk[m]
            ok = B[jj, kk] >= 0
            # closure: d_ij + d_jk + d_ki == 0
            clo = np.all(D[i, jj] + D[jj, kk] - D[i, kk] == 0, axis=-1)
            sel = ok & clo
            jj, kk = jj[sel], kk[sel]
            bij, bik, bjk = B[i, jj], B[i, kk], B[jj, kk]
            for a, b_, c in ((bij, bik, bjk), (bik, bij, bjk),      # centre i
                             (bij, bjk, bik), (bjk, bij, bik),      # centre j
                             (bik, bjk, bij), (bjk, bik, bij)):     # centre k
                np.add.at(H, (a, b_, c), 1)
    return H


def fcc_vectors(a_u: int, reach: float) -> np.ndarray:
    """FCC lattice vectors (a/2)(i, j, k), i + j + k even, 0 < |v| < reach."""
    h = a_u // 2
    m = int(np.ceil(reach / h)) + 1
    r = np.arange(-m, m + 1)
    I, J, K = np.meshgrid(r, r, r, indexing="ij")
    v = np.stack([I, J, K], -1).reshape(-1, 3)
    v = v[(v.sum(-1) % 2) == 0] * h
    n2 = (v * v).sum(-1)
    return v[(n2 > 0) & (n2 < reach * reach)]


def diamond_vectors(a_u: int, reach: float) -> np.ndarray:
    """Neighbour vectors of an A site of the diamond lattice (FCC + basis
    (a/4)(1,1,1)); B sites see the inverted set."""
    q = a_u // 4
    f = fcc_vectors(a_u, reach + 2 * a_u)
    f0 = np.concatenate([f, np.zeros((1, 3), dtype=f.dtype)])
    cross = f0 + np.array([q, q, q])
    v = np.concatenate([f, cross])
    n2 = (v * v).sum(-1)
    return v[(n2 > 0) & (n2 < reach * reach)]


def lattice_full(vectors: np.ndarray, n_sites: int, rmax: float, nbins: int,
                 nbins_third: int | None = None) -> np.ndarray:
    """N x #{(u, v): u != v, |u|, |v| < rmax, |v - u| < nbins_third rmax /
    nbins} binned (ordered)."""
    nc = nbins_third or nbins
    v = np.asarray(vectors, dtype=np.int64)
    bv = _bins_np((v * v).sum(-1), rmax, nbins)
    keep = bv >= 0
    v, bv = v[keep], bv[keep]
    D = v[None, :, :] - v[:, None, :]                   # D[p, q] = v_q - v_p
    bd = _bins_np((D * D).sum(-1), rmax, nbins, nc)
    P, Q = np.meshgrid(np.arange(len(v)), np.arange(len(v)), indexing="ij")
    m = (P != Q) & (bd >= 0)
    H = np.zeros((nbins, nbins, nc), dtype=np.uint64)
    np.add.at(H, (bv[P[m]], bv[Q[m]], bd[m]), 1)
    return H * np.uint64(n_sites)


def permutations_of(H: np.ndarray):
    for p in itertools.permutations(range(3)):
        yield p, np.transpose(H, p)


def brute_half(frames, box, rmax: float, nbins: int, nbins_third: int | None = None) -> dict:
    """Unordered triplets counted straight into the half layout: for every
    centre i and every pair j < k (both != i) with |d_ij|, |d_ik| < rmax and
    the third side d_ik - d_ij (no second minimum image) inside the
    nbins_third bins, key (min(b_ij, b_ik), max(b_ij, b_ik), b_jk) gains 1.
    No full histogram and no fold: a different route from the oracle's."""
    nc = nbins_third or nbins
    fr = np.asarray(frames, dtype=np.int64)
    F, _, N = fr.shape
    out: dict[tuple[int, int, int], int] = {}
    cache: dict[int, int] = {}
    cache3: dict[int, int] = {}

    def b(s):
        if s not in cache:
            cache[s] = frac_bin(s, rmax, nbins)
        return cache[s]

    def b3(s):
        if s not in cache3:
            cache3[s] = frac_bin_n(s, rmax, nbins, nc)
        return cache3[s]

    for f in range(F):
        P = [tuple(int(fr[f, d, a]) for d in range(3)) for a in range(N)]
        for i in range(N):
            near = []
            for j in range(N):
                if j == i:
                    continue
                d = [min_image(P[j][a] - P[i][a], box[a]) for a in range(3)]
                bj = b(sum(x * x for x in d))
                if bj >= 0:
                    near.append((d, bj))
            for x in range(len(near)):
                for y in range(x + 1, len(near)):
                    (dj, bj), (dk, bk) = near[x], near[y]
                    c = b3(sum((dk[a] - dj[a]) ** 2 for a in range(3)))
                    if c < 0:
                        continue
                    key = (min(bj, bk), max(bj, bk), c)
                    out[key] = out.get(key, 0) + 1
    return out


def half_order(nbins: int, nc: int) -> list:
    """The half layout's bins in storage order, listed one by one: rows
    lo = 0.. with columns hi = lo..nbins-1, each with nc third-side bins."""
    return [(lo, hi, c) for lo in range(nbins) for hi in range(lo, nbins) for c in range(nc)]
