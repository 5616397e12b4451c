"""g3 oracle -- TEST INFRASTRUCTURE ONLY.

A plain CPU statement of the triplet correlation histogram (Sec. 3.3, Eq. 3
and the triplet conditions after it) used to check the HIP library.  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the library never does, and the two share no code.

The arithmetic lives in ``g3_oracle.c`` (built into ``liboracle.so`` next to
this file by :func:`build`); this module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "g3_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-D_GNU_SOURCE", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.g3o_thresholds.argtypes = [C.c_double, C.c_int, P]
        L.g3o_thresholds.restype = C.c_int
        L.g3o_bin.argtypes = [C.c_uint64, P, C.c_int]
        L.g3o_bin.restype = C.c_int
        L.g3o_hist_full.argtypes = [P, C.c_int, C.c_int, P, C.c_double, C.c_int, P, C.c_int,
                                    P, C.c_int]
        L.g3o_hist_full.restype = C.c_int
        L.g3o_hist_full3.argtypes = [P, C.c_int, C.c_int, P, C.c_double, C.c_int, C.c_int, P,
                                     C.c_int, P, C.c_int]
        L.g3o_hist_full3.restype = C.c_int
        L.g3o_thresholds_n.argtypes = [C.c_double, C.c_int, C.c_int, P]
        L.g3o_thresholds_n.restype = C.c_int
        L.g3o_half_len3.argtypes = [C.c_int, C.c_int]
        L.g3o_half_len3.restype = C.c_size_t
        L.g3o_fold_half3.argtypes = [P, C.c_int, C.c_int, P]
        L.g3o_fold_half3.restype = C.c_long
        L.g3o_W_table3.argtypes = [C.c_int, C.c_int, C.c_double, P]
        L.g3o_W_table3.restype = None
        L.g3o_normalize3.argtypes = [P, C.c_int, C.c_int, C.c_int, P, C.c_int64, C.c_int64, P, P]
        L.g3o_normalize3.restype = None
        L.g3o_pair_hist.argtypes = [P, C.c_int, C.c_int, P, C.c_double, C.c_int, P, C.c_int]
        L.g3o_pair_hist.restype = C.c_int
        L.g3o_fold_half.argtypes = [P, C.c_int, P]
        L.g3o_fold_half.restype = C.c_long
        L.g3o_half_len.argtypes = [C.c_int]
        L.g3o_half_len.restype = C.c_size_t
        L.g3o_W_box.argtypes = [C.c_double] * 6
        L.g3o_W_box.restype = C.c_double
        L.g3o_W_table.argtypes = [C.c_int, C.c_double, P]
        L.g3o_W_table.restype = None
        L.g3o_normalize.argtypes = [P, C.c_int, C.c_int, P, C.c_int64, C.c_int64, P, P]
        L.g3o_normalize.restype = None
        L.g3o_normalize_pairs.argtypes = [P, C.c_int, C.c_double, C.c_int64, C.c_int64, P, P]
        L.g3o_normalize_pairs.restype = None
        L.g3o_max_threads.argtypes = []
        L.g3o_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def thresholds_n(rmax: float, nbins: int, count: int) -> np.ndarray:
    """thr[b] = ceil((b rmax / nbins)^2) for b = 0..count."""
    thr = np.zeros(count + 1, dtype=np.uint64)
    if lib().g3o_thresholds_n(float(rmax), int(nbins), int(count), _p(thr)):
        raise ValueError("oracle rejected the arguments")
    return thr


def thresholds(rmax: float, nbins: int) -> np.ndarray:
    thr = np.zeros(nbins + 1, dtype=np.uint64)
    if lib().g3o_thresholds(float(rmax), int(nbins), _p(thr)):
        raise ValueError("bad rmax/nbins")
    return thr


def bin_of(s: int, thr: np.ndarray) -> int:
    thr = np.ascontiguousarray(thr, dtype=np.uint64)
    return int(lib().g3o_bin(int(s), _p(thr), len(thr) - 1))


def _frames(frames) -> np.ndarray:
    fr = np.ascontiguousarray(frames, dtype=np.int32)
    assert fr.ndim == 3 and fr.shape[1] == 3
    return fr


def hist_full(frames, box, rmax: float, nbins: int, n_threads: int = 0,
              centres=None, nbins_third: int | None = None) -> np.ndarray:
    """H_full[b_ij][b_ik][b_jk] over ordered (j, k); shape (nbins, nbins,
    nbins_third) uint64 (third side in nbins_third bins of width rmax/nbins)."""
    nc = int(nbins_third or nbins)
    fr = _frames(frames)
    bx = np.ascontiguousarray(box, dtype=np.int32)
    H = np.zeros(nbins * nbins * nc, dtype=np.uint64)
    if centres is not None:
        ct = np.ascontiguousarray(centres, dtype=np.int32)
        cp, ncen = _p(ct), len(ct)
    else:
        ct, cp, ncen = None, None, 0
    rc = lib().g3o_hist_full3(_p(fr), fr.shape[0], fr.shape[2], _p(bx), float(rmax), int(nbins),
                              nc, _p(H), int(n_threads), cp, ncen)
    if rc:
        raise ValueError("oracle rejected the arguments")
    return H.reshape(nbins, nbins, nc)


def fold_half(full: np.ndarray) -> tuple[np.ndarray, int]:
    """(H_half flat, number of symmetry violations)."""
    nbins, nc = full.shape[0], full.shape[2]
    f = np.ascontiguousarray(full, dtype=np.uint64).reshape(-1)
    half = np.zeros(lib().g3o_half_len3(nbins, nc), dtype=np.uint64)
    bad = lib().g3o_fold_half3(_p(f), nbins, nc, _p(half))
    return half, int(bad)


def hist(frames, box, rmax: float, nbins: int, layout: int, n_threads: int = 0,
         centres=None, nbins_third: int | None = None) -> np.ndarray:
    """Flat histogram in the library's layout (0 = half, 1 = full)."""
    full = hist_full(frames, box, rmax, nbins, n_threads, centres, nbins_third)
    if layout == 1:
        return full.reshape(-1)
    half, bad = fold_half(full)
    if bad:
        raise AssertionError(f"oracle H_full lacks its symmetry at {bad} bins")
    return half


def pair_hist(frames, box, rmax: float, nbins: int, n_threads: int = 0) -> np.ndarray:
    fr = _frames(frames)
    bx = np.ascontiguousarray(box, dtype=np.int32)
    H2 = np.zeros(nbins, dtype=np.uint64)
    if lib().g3o_pair_hist(_p(fr), fr.shape[0], fr.shape[2], _p(bx), float(rmax), int(nbins),
                           _p(H2), int(n_threads)):
        raise ValueError("oracle rejected the arguments")
    return H2


def W_box(a0, a1, b0, b1, c0, c1) -> float:
    return float(lib().g3o_W_box(a0, a1, b0, b1, c0, c1))


def W_table(nbins: int, dr: float, nbins_third: int | None = None) -> np.ndarray:
    nc = int(nbins_third or nbins)
    W = np.zeros(nbins * nbins * nc, dtype=np.float64)
    lib().g3o_W_table3(int(nbins), nc, float(dr), _p(W))
    return W.reshape(nbins, nbins, nc)


def normalize(H: np.ndarray, layout: int, nbins: int, rmax: float, n_frames: int,
              n_atoms: int, box, nbins_third: int | None = None) -> np.ndarray:
    nc = int(nbins_third or nbins)
    W = np.ascontiguousarray(W_table(nbins, rmax / nbins, nc).reshape(-1))
    Hc = np.ascontiguousarray(H, dtype=np.uint64).reshape(-1)
    out = np.zeros(Hc.shape[0], dtype=np.float64)
    bx = np.ascontiguousarray(box, dtype=np.int32)
    lib().g3o_normalize3(_p(Hc), int(layout == 1), int(nbins), nc, _p(W), int(n_frames),
                         int(n_atoms), _p(bx), _p(out))
    return out


def normalize_pairs(H2: np.ndarray, nbins: int, rmax: float, n_frames: int, n_atoms: int,
                    box) -> np.ndarray:
    h = np.ascontiguousarray(H2, dtype=np.uint64).reshape(-1)
    out = np.zeros(int(nbins), dtype=np.float64)
    bx = np.ascontiguousarray(box, dtype=np.int32)
    lib().g3o_normalize_pairs(_p(h), int(nbins), float(rmax), int(n_frames), int(n_atoms),
                              _p(bx), _p(out))
    return out


def superposition_full(g3_full: np.ndarray, g2: np.ndarray) -> np.ndarray:
    """Kirkwood superposition test: g3(a,b,c) / (g2(a) g2(b) g2(c)) on the
    full nbins^3 array, 0 where the product is 0 (angle-resolved motivation
    of Sec. 3.3).  Plain loops over bins."""
    G = np.asarray(g3_full, dtype=np.float64)
    nb = G.shape[0]
    out = np.zeros_like(G)
    for a in range(nb):
        for b in range(nb):
            for c in range(nb):
                d = g2[a] * g2[b] * g2[c]
                out[a, b, c] = G[a, b, c] / d if d > 0 else 0.0
    return out


def isosceles_angle(a: int, c: int) -> float:
    """Apex angle of the isosceles triangle with both sides at the centre of
    bin a and the third side at the centre of bin c (law of cosines), or -1
    if no such triangle exists."""
    import math
    r, t = a + 0.5, c + 0.5
    if t > 2 * r:
        return -1.0
    return math.acos(1.0 - t * t / (2.0 * r * r))


def max_threads() -> int:
    return int(lib().g3o_max_threads())
