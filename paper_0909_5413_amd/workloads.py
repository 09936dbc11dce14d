"""Seeded synthetic workloads: jittered square lattices, Gaussian-vortex data.

This module only draws inputs.  It holds none of the interpolation method's
arithmetic, so both the GPU path and the CPU oracle can be fed from it.

The point sets follow the paper's experiments (Section 3.1): points on a
square lattice, optionally shifted by a random amount to make them
quasi-scattered.  Here the lattice is cell-centred on [-1, 1]^2 with spacing
h = 2 / n_side and every coordinate is shifted by an independent uniform
offset in [-0.1 h, +0.1 h].  The Gaussian width is fixed through the overlap
ratio h / sigma, the quantity the paper's convergence study varies
(Section 3.2), and the matvec cutoff is r_c = 6 sigma.

The interpolated data is a normalised Gaussian vortex
f(x) = exp(-|x|^2 / r0^2) / (pi r0^2), the kind of field the paper's target
application (vortex particle methods, Section 1) interpolates.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 5413


@dataclass(frozen=True)
class Workload:
    name: str
    n_side: int
    h_over_sigma: float = 0.8
    jitter: float = 0.1          # fraction of h, uniform +-jitter*h per coordinate
    r0: float = 0.2              # Gaussian-vortex core radius of the data
    rtol: float = 1e-10
    seed: int = SEED_BASE
    cutoff_sigmas: float = 6.0
    overlap: int = 1
    notes: str = field(default="", compare=False)

    @property
    def n(self) -> int:
        return self.n_side * self.n_side

    @property
    def h(self) -> float:
        return 2.0 / self.n_side

    @property
    def sigma(self) -> float:
        return self.h / self.h_over_sigma

    @property
    def cutoff(self) -> float:
        return self.cutoff_sigmas * self.sigma

    def points(self) -> np.ndarray:
        return jittered_lattice(self.n_side, self.jitter, self.seed)

    def values(self, pts: np.ndarray | None = None) -> np.ndarray:
        if pts is None:
            pts = self.points()
        return gaussian_vortex(pts, self.r0)


def jittered_lattice(n_side: int, jitter: float = 0.1, seed: int = SEED_BASE,
                     lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """n_side^2 points, row-major (index = iy * n_side + ix), shape (N, 2) float64.

    Lattice x_k = lo + (k + 1/2) h with h = (hi - lo) / n_side, each coordinate
    shifted by an independent U(-jitter*h, +jitter*h) drawn from PCG64(seed).
    """
    h = (hi - lo) / n_side
    k = np.arange(n_side, dtype=np.float64)
    c = lo + (k + 0.5) * h
    xx, yy = np.meshgrid(c, c, indexing="xy")        # yy varies along rows
    pts = np.stack([xx.ravel(), yy.ravel()], axis=1)
    if jitter:
        rng = np.random.default_rng(seed)
        pts = pts + rng.uniform(-jitter * h, jitter * h, size=pts.shape)
    return np.ascontiguousarray(pts, dtype=np.float64)


def gaussian_vortex(pts: np.ndarray, r0: float = 0.2) -> np.ndarray:
    """f(x) = exp(-|x|^2 / r0^2) / (pi r0^2), unit total circulation."""
    r2 = pts[:, 0] ** 2 + pts[:, 1] ** 2
    return np.exp(-r2 / (r0 * r0)) / (np.pi * r0 * r0)


def franke(pts: np.ndarray) -> np.ndarray:
    """Franke's test function for 2-D scattered-data fitting (the paper's test
    data, Section 3.1), meant for points in [0, 1]^2."""
    x, y = pts[:, 0], pts[:, 1]
    return (0.75 * np.exp(-((9 * x - 2) ** 2 + (9 * y - 2) ** 2) / 4)
            + 0.75 * np.exp(-((9 * x + 1) ** 2) / 49 - (9 * y + 1) / 10)
            + 0.5 * np.exp(-((9 * x - 7) ** 2 + (9 * y - 3) ** 2) / 4)
            - 0.2 * np.exp(-(9 * x - 4) ** 2 - (9 * y - 7) ** 2))


def unit_square_lattice(n_side: int, h_over_sigma: float, jitter: float = 0.1, seed: int = SEED_BASE):
    """The paper's layout (Section 3.1): a jittered n_side^2 lattice on [0, 1]^2
    (cell-centred, spacing h = 1 / n_side), and sigma = h / (h/sigma)."""
    pts = jittered_lattice(n_side, jitter, seed, lo=0.0, hi=1.0)
    return pts, (1.0 / n_side) / h_over_sigma


def random_weights(n: int, seed: int) -> np.ndarray:
    """w ~ U(-1, 1), float64, for matvec micro-benchmarks and parity tests."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


def staggered_lattice(n_side: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Evaluation points midway between lattice nodes: (n_side - 1)^2 points."""
    h = (hi - lo) / n_side
    c = lo + (np.arange(n_side - 1, dtype=np.float64) + 1.0) * h
    xx, yy = np.meshgrid(c, c, indexing="xy")
    return np.ascontiguousarray(np.stack([xx.ravel(), yy.ravel()], axis=1))


def evaluation_targets(pts: np.ndarray, cutoff: float, seed: int = 41):
    """Targets for the interpolant off the nodes, and how many of them (the
    last ones) lie farther than the cutoff from every node: five nodes, 60
    points midway between consecutive nodes, 80 uniform points in the nodes'
    bounding box, points 0.3 and 0.9 cutoffs outside each edge and corner of
    that box (3 per side or corner and distance, 48 in all), and 4 points
    more than a cutoff away from the box."""
    rng = np.random.default_rng(seed)
    lo, hi = pts.min(axis=0), pts.max(axis=0)
    mid = 0.5 * (lo + hi)
    out = [pts[:5], 0.5 * (pts[:60] + pts[1:61]), rng.uniform(lo, hi, (80, 2))]
    near = []
    for d in (0.3, 0.9):
        for sx in (-1, 0, 1):
            for sy in (-1, 0, 1):
                if sx == 0 and sy == 0:
                    continue
                for t in (0.1, 0.5, 0.85):
                    base = lo + t * (hi - lo)
                    x = lo[0] - d * cutoff if sx < 0 else hi[0] + d * cutoff if sx > 0 else base[0]
                    y = lo[1] - d * cutoff if sy < 0 else hi[1] + d * cutoff if sy > 0 else base[1]
                    near.append((x, y))
    out.append(np.array(near))
    far = np.array([(hi[0] + 1.5 * cutoff, mid[1]), (lo[0] - 2.0 * cutoff, lo[1] - 2.0 * cutoff),
                    (mid[0], hi[1] + 1.01 * cutoff), (50.0, -40.0)])
    out.append(far)
    return np.ascontiguousarray(np.concatenate(out)), len(far)


# The workloads, sized like the paper's lattice runs (Sections 3 and 4).
MINI = Workload("mini", 44, 0.8, rtol=1e-10, seed=SEED_BASE + 100,
                notes="44x44 lattice, N=1936: small enough for dense checks")
C0 = Workload("c0", 100, 0.8, rtol=1e-10, seed=SEED_BASE + 0,
              notes="N=10,000, h=0.02, GMRES(30) to 1e-10")
C1 = Workload("c1", 1000, 0.8, rtol=1e-12, seed=SEED_BASE + 1,
              notes="N=1,000,000, h=0.002, GMRES(30) to 1e-12")
C2 = {r: Workload(f"c2_{r}", 2048, r, rtol=1e-12, seed=SEED_BASE + 2,
                  notes="N=4,194,304 mixed-precision sweep")
      for r in (0.6, 0.8, 1.0)}
C4 = Workload("c4", 7072, 0.8, rtol=1e-14, seed=SEED_BASE + 4,
              notes="N=50,013,184, largest single problem")

WORKLOADS = {w.name: w for w in (MINI, C0, C1, C4, *C2.values())}


def sub_lattice(w: Workload, n_side: int) -> Workload:
    """A smaller lattice with the same spacing ratio, jitter and cutoff rule."""
    return Workload(f"{w.name}_sub{n_side}", n_side, w.h_over_sigma, w.jitter, w.r0,
                    w.rtol, w.seed, w.cutoff_sigmas, w.overlap)


def serving_requests(k: int, seed_base: int = SEED_BASE * 1000, n_lo: float = 1e3,
                     n_hi: float = 1e6, hs_lo: float = 0.6, hs_hi: float = 1.0,
                     r0_lo: float = 0.1, r0_hi: float = 0.4, rtol: float = 1e-12) -> list:
    """A stream of k interpolation requests: request i draws, from
    default_rng(seed_base + i), N log-uniform in [n_lo, n_hi] (n_side =
    round(sqrt(N))), h/sigma uniform in [hs_lo, hs_hi] and the data's core
    radius r0 uniform in [r0_lo, r0_hi]; its points use the same seed."""
    out = []
    for i in range(k):
        rng = np.random.default_rng(seed_base + i)
        n = float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        hs = float(rng.uniform(hs_lo, hs_hi))
        r0 = float(rng.uniform(r0_lo, r0_hi))
        side = max(int(round(np.sqrt(n))), 4)
        out.append(Workload(f"req{i}", side, hs, r0=r0, rtol=rtol, seed=seed_base + i))
    return out
