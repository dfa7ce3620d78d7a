"""Seeded synthetic workloads for the short-range TreePM gravity solver.

This module only draws inputs: particle positions, masses, softening lengths,
solver parameters, active subsets and cotangent weights.  It holds none of the
solver's arithmetic, so both the HIP path and the CPU oracle can be fed from it.

The paper's own workloads (the Magneticum dark-matter-only box of Sec. 3.1 and
the Dianoga zoom-in clusters of Secs. 3.3-3.4) are not available; the recipes
below stand in for them:

* a uniform periodic box stands in for the "very homogeneous" early-time
  initial conditions of the chip-to-chip scaling runs (Sec. 4.1);
* Plummer spheres on a uniform background stand in for late-time clustered
  haloes (Sec. 3.1, and the caveat on more clustered conditions in Sec. 4.1);
* a dense high-resolution sphere inside a heavier perturbed-grid background
  stands in for a zoom-in cluster re-simulation (Secs. 3.3-3.4).

All draws use numpy's PCG64 ``default_rng(seed)`` in a fixed order, and every
particle set is returned in a seeded random order so that the key sort has real
work to do.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Gadget-style TreePM split defaults: r_s = ASMTH * L / N_mesh, r_cut = RCUT * r_s.
ASMTH = 1.25
RCUT = 4.5
# The softening of every configuration is one thirtieth of the mean spacing.
SOFT_FRACTION = 1.0 / 30.0


@dataclass
class Workload:
    """One synthetic particle set plus the solver parameters it is run with."""

    name: str
    pos: np.ndarray                 # (N, 3) float64, may lie outside [0, box)
    mass: np.ndarray                # (N,) float64
    eps: np.ndarray                 # (N,) float64 Plummer-equivalent softening
    box: float = 1.0
    G: float = 1.0
    r_s: float = 0.0
    r_cut: float = 0.0
    theta: float = 0.5
    criterion: str = "bh"           # "bh" or "relative"
    alpha: float = 0.0
    active: Optional[np.ndarray] = None   # (n_active,) int32 input indices, or None
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def params(self, precision: str = "fp64") -> dict:
        return dict(G=self.G, r_s=self.r_s, r_cut=self.r_cut, theta=self.theta,
                    criterion=self.criterion, alpha=self.alpha, precision=precision)


def split_scales(n_mesh: int, box: float = 1.0):
    """PM split scale and short-range cutoff for a mesh of n_mesh cells per side."""
    r_s = ASMTH * box / n_mesh
    return r_s, RCUT * r_s


def _plummer_offsets(rng, count: int, a: float) -> np.ndarray:
    """Offsets of `count` points drawn from an untruncated Plummer sphere of scale a."""
    x = rng.random(count)
    # Inverse of the Plummer cumulative mass profile M(<r)/M = r^3 / (r^2 + a^2)^(3/2).
    with np.errstate(divide="ignore"):
        radius = a / np.sqrt(np.power(x, -2.0 / 3.0) - 1.0)
    radius = np.where(np.isfinite(radius), radius, 0.0)
    direction = rng.standard_normal((count, 3))
    direction /= np.linalg.norm(direction, axis=1, keepdims=True)
    return direction * radius[:, None]


def _largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    share = weights / weights.sum() * total
    counts = np.floor(share).astype(np.int64)
    rest = total - int(counts.sum())
    frac = share - counts
    # Largest fractional parts first; ties go to the lower index (stable sort).
    order = np.argsort(-frac, kind="stable")
    counts[order[:rest]] += 1
    return counts


def clustered_positions(rng, n: int, n_spheres: int, cluster_fraction: float = 0.7,
                        a_min: float = 0.002, a_max: float = 0.02,
                        pareto_alpha: float = 1.5) -> np.ndarray:
    """Plummer spheres (Pareto-distributed memberships) on a uniform background."""
    n_cl = int(np.floor(cluster_fraction * n))
    n_bg = n - n_cl
    weights = 1.0 + rng.pareto(pareto_alpha, n_spheres)
    counts = _largest_remainder(weights, n_cl)
    centres = rng.random((n_spheres, 3))
    scales = np.exp(rng.uniform(np.log(a_min), np.log(a_max), n_spheres))
    parts = []
    for c, a, k in zip(centres, scales, counts):
        if k:
            parts.append(c + _plummer_offsets(rng, int(k), float(a)))
    parts.append(rng.random((n_bg, 3)))
    pos = np.concatenate(parts, axis=0)
    pos = np.mod(pos, 1.0)
    return pos[rng.permutation(n)]


def uniform(n: int, seed: int, n_mesh: Optional[int] = None, name: str = "uniform") -> Workload:
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    side = round(n ** (1.0 / 3.0))
    n_mesh = n_mesh or 2 * side
    r_s, r_cut = split_scales(n_mesh)
    eps = np.full(n, SOFT_FRACTION / side)
    return Workload(name, pos, np.full(n, 1.0 / n), eps, r_s=r_s, r_cut=r_cut)


def clustered(n: int, seed: int, n_spheres: int, n_mesh: Optional[int] = None,
              name: str = "clustered") -> Workload:
    rng = np.random.default_rng(seed)
    pos = clustered_positions(rng, n, n_spheres)
    side = round(n ** (1.0 / 3.0))
    n_mesh = n_mesh or 2 * side
    r_s, r_cut = split_scales(n_mesh)
    eps = np.full(n, SOFT_FRACTION / side)
    return Workload(name, pos, np.full(n, 1.0 / n), eps, r_s=r_s, r_cut=r_cut)


# --- the five named configurations ------------------------------------------------

def uniform_32k() -> Workload:
    """32^3 equal-mass particles, uniform i.i.d., PM mesh 64^3, FP64 reference case."""
    return uniform(32 ** 3, seed=1, n_mesh=64, name="uniform_32k")


def clustered_262k() -> Workload:
    """64^3 particles, 70% in 200 Plummer spheres, PM mesh 128^3."""
    return clustered(64 ** 3, seed=2, n_spheres=200, n_mesh=128, name="clustered_262k")


def clustered_2m_active() -> Workload:
    """128^3 particles in 400 spheres, relative opening, random 10% active subset."""
    n = 128 ** 3
    w = clustered(n, seed=3, n_spheres=400, n_mesh=256, name="clustered_2m_active")
    rng = np.random.default_rng(103)
    w.active = np.sort(rng.choice(n, 209_715, replace=False)).astype(np.int32)
    w.criterion = "relative"
    w.alpha = 0.005
    w.theta = 0.7
    return w


def deep_chains(levels: int = 25) -> Workload:
    """A chain of nested cells in every cell of the 8^3 grid: at each of `levels`
    levels one particle at the centre of seven octants and the eighth octant
    refined again, down to octree level 27 (exact dyadic positions, 93,696
    particles for 25 levels).  Sorted, the particles of any 512-particle run end
    inside a chain, so up to 25 nested nodes reach past the run's end, each with
    seven particle children; the tree is 28 nodes deep."""
    pts = []
    octs = np.array([[(o >> 0) & 1, (o >> 1) & 1, (o >> 2) & 1] for o in range(8)], dtype=np.float64)
    for ix in range(8):
        for iy in range(8):
            for iz in range(8):
                c = np.array([ix, iy, iz], dtype=np.float64) / 8.0
                s = 1.0 / 8.0
                for _ in range(levels):
                    pts.append(c + s * (0.25 + 0.5 * octs[1:]))
                    s *= 0.5
                pts.append(c + s * (0.25 + 0.5 * octs))
    pos = np.concatenate(pts)
    n = pos.shape[0]
    w = Workload("deep_chains", pos, np.full(n, 1.0 / n), np.full(n, 1 / 600.0))
    w.r_s, w.r_cut = split_scales(48)
    return w


def adjoint_weights(n: int, seed: int = 104) -> np.ndarray:
    """Cotangent w_i ~ N(0, 1)^3 of the loss L = sum_i w_i . a_i."""
    return np.random.default_rng(seed).standard_normal((n, 3))


def fd_subset(n: int, count: int = 4096, seed: int = 204) -> np.ndarray:
    return np.sort(np.random.default_rng(seed).choice(n, count, replace=False)).astype(np.int64)


def clustered_4k_for_gradient() -> Workload:
    """4096 particles from the clustered recipe with the 262k case's split and softening."""
    base = clustered_262k()
    w = clustered(4096, seed=304, n_spheres=200, name="clustered_4k_grad")
    w.r_s, w.r_cut, w.eps = base.r_s, base.r_cut, np.full(4096, base.eps[0])
    return w


def zoom(n_hi: int, bg_side: int, seed: int = 5, name: str = "zoom") -> Workload:
    """High-resolution sphere (radius 0.1) inside a perturbed-grid background.

    Background particles weigh 64 high-resolution masses, the total mass is 1 and
    the high-resolution softening is a quarter of the background one.
    """
    rng = np.random.default_rng(seed)
    radius = 0.1 * np.cbrt(rng.random(n_hi))
    direction = rng.standard_normal((n_hi, 3))
    direction /= np.linalg.norm(direction, axis=1, keepdims=True)
    hi = 0.5 + direction * radius[:, None]
    g = (np.arange(bg_side) + 0.5) / bg_side
    gx, gy, gz = np.meshgrid(g, g, g, indexing="ij")
    bg = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    bg = bg + rng.normal(0.0, 0.1 / bg_side, bg.shape)
    n_bg = bg.shape[0]
    m = 1.0 / (n_hi + 64 * n_bg)
    pos = np.concatenate([hi, bg])
    mass = np.concatenate([np.full(n_hi, m), np.full(n_bg, 64 * m)])
    eps_bg = 1.0 / 3840.0
    eps = np.concatenate([np.full(n_hi, eps_bg / 4), np.full(n_bg, eps_bg)])
    order = rng.permutation(n_hi + n_bg)
    r_s, r_cut = split_scales(256)
    w = Workload(name, np.mod(pos[order], 1.0), mass[order], eps[order], r_s=r_s, r_cut=r_cut)
    w.extra["vel"] = np.zeros_like(w.pos)
    w.extra["n_steps"] = 8
    w.extra["dt"] = 1e-3
    w.extra["loss_w"] = np.random.default_rng(105).standard_normal(w.pos.shape)
    return w


def zoom_6m() -> Workload:
    """4,194,304 high-resolution particles in 2,097,152 background ones (128^3 grid)."""
    return zoom(4_194_304, 128, name="zoom_6m")


def zoom_small() -> Workload:
    """The zoom-in recipe scaled down 64-fold (65,536 + 32^3 particles)."""
    return zoom(65_536, 32, name="zoom_98k")


CONFIGS = {
    "uniform_32k": uniform_32k,
    "clustered_262k": clustered_262k,
    "clustered_2m_active": clustered_2m_active,
    "zoom_6m": zoom_6m,
}
