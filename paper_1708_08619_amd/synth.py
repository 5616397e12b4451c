"""Seeded synthetic trajectories for the g3 triplet histogram.

This module only *draws* inputs: integer positions in an orthorhombic box,
shaped like the paper's workloads (a Lennard-Jones-like fluid and water-like
oxygen sites, Sec. 2.1; the g3 runs of Table 2).  It holds none of the
method's arithmetic (no distances, no binning), so both the CPU oracle and the
HIP path may consume what it produces.

Conventions
-----------
* Frames are int32 arrays of shape ``[n_frames, 3, n_atoms]`` (structure of
  arrays per frame, the flat per-frame layout the paper uses for its device
  arrays), every coordinate in ``[0, L_d)``.
* Positions are drawn in real units, rounded to the nearest integer unit and
  wrapped by integer ``mod L_d``.
* Every draw is reproducible from ``numpy.random.SeedSequence(seed)``; frames
  (and systems) get their own ``spawn()``-ed child streams.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 20170828  # configs use SEED_BASE + config number

# Fixed-point units: LJ systems use sigma/4096, water-like systems 2^-16 nm.
LJ_UNIT_PER_SIGMA = 4096
WATER_UNIT_PER_NM = 65536


def _rng(seed_seq: np.random.SeedSequence) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_seq))


def _as_frames(pos: np.ndarray, box) -> np.ndarray:
    """[F, N, 3] int64 -> wrapped [F, 3, N] int32."""
    box = np.asarray(box, dtype=np.int64)
    pos = np.mod(pos, box[None, None, :])
    return np.ascontiguousarray(pos.transpose(0, 2, 1)).astype(np.int32)


def uniform_frames(n_atoms: int, box, n_frames: int, seed) -> np.ndarray:
    """Ideal gas: i.i.d. uniform integer positions in [0, L_d)."""
    ss = np.random.SeedSequence(seed)
    out = np.empty((n_frames, 3, n_atoms), dtype=np.int32)
    for f, child in enumerate(ss.spawn(n_frames)):
        g = _rng(child)
        for d in range(3):
            out[f, d] = g.integers(0, int(box[d]), size=n_atoms, dtype=np.int64)
    return out


def fcc_sites(n_cells: int, a_u: int) -> np.ndarray:
    """Integer sites of an n^3 FCC lattice of cubic cell a_u (a_u even)."""
    assert a_u % 2 == 0
    h = a_u // 2
    basis = np.array([[0, 0, 0], [0, h, h], [h, 0, h], [h, h, 0]], dtype=np.int64)
    g = np.arange(n_cells, dtype=np.int64) * a_u
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    return (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)


def diamond_sites(n_cells: int, a_u: int) -> np.ndarray:
    """Integer sites of an n^3 diamond lattice of cubic cell a_u (a_u % 4 == 0)."""
    assert a_u % 4 == 0
    f = fcc_sites(n_cells, a_u)
    q = a_u // 4
    return np.concatenate([f, f + np.array([q, q, q], dtype=np.int64)], axis=0)


def lattice_frames(sites: np.ndarray, n_atoms: int, box, jitter_sd_u: float,
                   n_frames: int, seed) -> np.ndarray:
    """Keep a seeded random subset of ``n_atoms`` lattice sites (the same for
    every frame) and add Gaussian jitter of sd ``jitter_sd_u`` units, redrawn
    per frame, rounded to the nearest unit and wrapped."""
    ss = np.random.SeedSequence(seed)
    pick_ss, frames_ss = ss.spawn(2)
    if n_atoms < len(sites):
        keep = np.sort(_rng(pick_ss).choice(len(sites), size=n_atoms, replace=False))
        sites = sites[keep]
    assert len(sites) == n_atoms
    pos = np.empty((n_frames, n_atoms, 3), dtype=np.int64)
    for f, child in enumerate(frames_ss.spawn(n_frames)):
        if jitter_sd_u > 0:
            j = np.rint(_rng(child).normal(0.0, jitter_sd_u, size=(n_atoms, 3))).astype(np.int64)
        else:
            j = 0
        pos[f] = sites + j
    return _as_frames(pos, box)


def smallest_cells(n_atoms: int, per_cell: int) -> int:
    n = 1
    while per_cell * n ** 3 < n_atoms:
        n += 1
    return n


def cubic_lattice_box(n_atoms: int, rho: float, unit_per_len: float, n_cells: int,
                      multiple: int) -> int:
    """Box edge in units for density rho, rounded to a multiple of
    ``multiple`` so that the lattice is integral."""
    L = (n_atoms / rho) ** (1.0 / 3.0) * unit_per_len
    return int(max(multiple, round(L / multiple) * multiple))


def jittered_fcc(n_atoms: int, rho: float, jitter_sigma: float, n_frames: int,
                 seed) -> tuple[np.ndarray, list[int]]:
    """Jittered FCC Lennard-Jones-like fluid in sigma/4096 units."""
    n = smallest_cells(n_atoms, 4)
    L = cubic_lattice_box(n_atoms, rho, LJ_UNIT_PER_SIGMA, n, 2 * n)
    sites = fcc_sites(n, L // n)
    frames = lattice_frames(sites, n_atoms, [L] * 3, jitter_sigma * LJ_UNIT_PER_SIGMA,
                            n_frames, seed)
    return frames, [L, L, L]


@dataclass
class Workload:
    """One system: frames plus the analysis parameters."""
    name: str
    frames: np.ndarray          # int32 [F, 3, N]
    box: list                   # 3 ints (units)
    rmax: float                 # units (binary64)
    nbins: int
    layout: int                 # 0 = half (lo <= hi), 1 = full
    meta: dict = field(default_factory=dict)

    @property
    def n_frames(self) -> int:
        return int(self.frames.shape[0])

    @property
    def n_atoms(self) -> int:
        return int(self.frames.shape[2])


HALF, FULL = 0, 1


def lj_small(kind: str = "fcc", n_frames: int = 10) -> Workload:
    """N=256 LJ-like fluid, rho=0.8 sigma^-3, rmax=2.5 sigma, 50 bins.

    ``kind='gas'``: uniform ideal gas; ``kind='fcc'``: FCC 4x4x4 with
    Gaussian jitter sd 0.1 sigma redrawn per frame."""
    N, rho = 256, 0.8
    n = smallest_cells(N, 4)                       # 4
    L = cubic_lattice_box(N, rho, LJ_UNIT_PER_SIGMA, n, 2 * n)
    box = [L, L, L]
    seed = SEED_BASE + 1
    if kind == "gas":
        frames = uniform_frames(N, box, n_frames, [seed, 0])
    else:
        frames = lattice_frames(fcc_sites(n, L // n), N, box, 0.1 * LJ_UNIT_PER_SIGMA,
                                n_frames, [seed, 1])
    return Workload(f"lj256_{kind}", frames, box, 2.5 * LJ_UNIT_PER_SIGMA, 50, FULL,
                    {"rho": rho, "unit": "sigma/4096"})


def water_like(n_frames: int = 100) -> Workload:
    """N=4096 oxygen-like sites at 33.4 nm^-3 on a jittered diamond lattice
    (sd 0.03 nm, redrawn per frame), unit 2^-16 nm, rmax=0.6 nm, 60 bins."""
    N, rho = 4096, 33.4
    n = smallest_cells(N, 8)                       # 8
    L = cubic_lattice_box(N, rho, WATER_UNIT_PER_NM, n, 4 * n)
    box = [L, L, L]
    frames = lattice_frames(diamond_sites(n, L // n), N, box, 0.03 * WATER_UNIT_PER_NM,
                            n_frames, [SEED_BASE + 2, 0])
    return Workload("water4096", frames, box, 0.6 * WATER_UNIT_PER_NM, 60, FULL,
                    {"rho": rho, "unit": "2^-16 nm"})


# Coarser unit for the paper-shape replays, so that L/2 stays within the
# 46340-unit limit of the third side for N up to 26880 at water density.
REPLAY_UNIT_PER_NM = 8192
PAPER_SHAPES = (6720, 13440, 26880)   # system sizes of the paper's Table 2 runs


def water_replay(n_atoms: int, n_frames: int = 10, nbins: int = 80) -> Workload:
    """Water-density oxygen-like sites (33.4 nm^-3) for a paper-shape replay
    of the g3 runs (Table 2: N = 6720, 13440, 26880, 10 frames): jittered
    diamond lattice (sd 0.03 nm, redrawn per frame, a seeded subset of the
    smallest 8 n^3 >= N sites), unit 2^-13 nm, the paper's geometry -- two
    sides below L/4, the third below L/2: rmax = L/4 with nbins bins and
    2 nbins third-side bins; full layout (the paper keeps the whole 3-D
    histogram).  The third-side bin count is meta["nbins_third"]."""
    rho = 33.4
    n = smallest_cells(n_atoms, 8)
    L = cubic_lattice_box(n_atoms, rho, REPLAY_UNIT_PER_NM, n, 4 * n)
    box = [L, L, L]
    frames = lattice_frames(diamond_sites(n, L // n), n_atoms, box, 0.03 * REPLAY_UNIT_PER_NM,
                            n_frames, [SEED_BASE + 6, n_atoms])
    return Workload(f"water_replay{n_atoms}", frames, box, L / 4.0, nbins, FULL,
                    {"rho": rho, "unit": "2^-13 nm", "nbins_third": 2 * nbins})


def uneven_batch(n_systems: int = 8, frames_per_system: int = 8) -> list[Workload]:
    """Batched case: systems with N log-uniform in [512, 32768], densities
    U(0.7, 0.9) sigma^-3, jittered FCC (sd 0.1 sigma), rmax 2.5 sigma, 50 bins."""
    ss = np.random.SeedSequence([SEED_BASE + 3, 0])
    out = []
    for s, child in enumerate(ss.spawn(n_systems)):
        g = _rng(child)
        N = int(round(math.exp(g.uniform(math.log(512), math.log(32768)))))
        rho = float(g.uniform(0.7, 0.9))
        frames, box = jittered_fcc(N, rho, 0.1, frames_per_system, [SEED_BASE + 3, 1, s])
        out.append(Workload(f"batch{s}_N{N}", frames, box, 2.5 * LJ_UNIT_PER_SIGMA, 50, FULL,
                            {"rho": rho}))
    return out


def lj_large(n_frames: int = 50) -> Workload:
    """N=65536 LJ-like fluid at rho=0.85 sigma^-3: FCC n=26 (70304 sites,
    seeded subset of 65536), jitter sd 0.15 sigma, rmax=3.0 sigma, 60 bins,
    half layout."""
    N, rho = 65536, 0.85
    frames, box = jittered_fcc(N, rho, 0.15, n_frames, [SEED_BASE + 4, 0])
    return Workload("lj65536", frames, box, 3.0 * LJ_UNIT_PER_SIGMA, 60, HALF,
                    {"rho": rho, "unit": "sigma/4096"})


def serving_requests(n_requests: int = 2000, rate_hz: float = 200.0, seed=None,
                     n_min: int = 1024, n_max: int = 65536, max_frames: int = 20):
    """Open-loop Poisson request stream: yields (arrival_s, Workload).

    Each request: frames ~ U{1..max_frames}, N log-uniform in [n_min, n_max],
    rmax in {2.0, 2.5, 3.0} sigma (dr = 0.05 sigma so nbins in {40, 50, 60}),
    rho ~ U(0.7, 0.9), jittered FCC sd 0.1 sigma.  Frames are drawn lazily."""
    ss = np.random.SeedSequence([SEED_BASE + 5, 0] if seed is None else seed)
    g = _rng(ss)
    t = 0.0
    for r in range(n_requests):
        t += float(g.exponential(1.0 / rate_hz))
        F = int(g.integers(1, max_frames + 1))
        N = int(round(math.exp(g.uniform(math.log(n_min), math.log(n_max)))))
        rm = float(g.choice([2.0, 2.5, 3.0]))
        rho = float(g.uniform(0.7, 0.9))
        yield t, {"id": r, "n_frames": F, "n_atoms": N, "rmax_sigma": rm, "rho": rho,
                  "seed": [SEED_BASE + 5, 1, r]}


def realize_request(req: dict) -> Workload:
    frames, box = jittered_fcc(req["n_atoms"], req["rho"], 0.1, req["n_frames"], req["seed"])
    rm = req["rmax_sigma"]
    return Workload(f"req{req['id']}", frames, box, rm * LJ_UNIT_PER_SIGMA,
                    int(round(rm / 0.05)), HALF, {"rho": req["rho"]})


def ideal_gas(n_atoms: int, box, n_frames: int, rmax: float, nbins: int,
              layout: int = FULL, seed=(SEED_BASE, 99)) -> Workload:
    return Workload(f"gas{n_atoms}", uniform_frames(n_atoms, box, n_frames, list(seed)),
                    list(box), float(rmax), int(nbins), layout)
