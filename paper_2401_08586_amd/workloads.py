"""Seeded synthetic particle sets shaped like the paper's neighbour-search workloads.

This module only draws inputs. It holds none of the search arithmetic, so the
CPU oracle and the HIP path can both take their inputs from it.

Shapes follow the paper's own synthetic cases:
  * lattices at spacing ds with smoothing length h = 1.2 ds, so the search
    radius is 2h = 2.4 ds (SPH method section, text after Eq. 3);
  * uniform random points in the unit domain, ds = (1/N)^(1/d)
    (Results, accuracy of FP16 neighbour search, text before Table 2);
  * one-million-particle cases (Results, efficiency section, Table 6).
Clustered sets and the serving mix are the batched and multi-simulation
workloads this library adds on top; they use the same radius rule.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class ParticleSet:
    """One search problem: positions [n, dim] float64 (row-major), box, cell size, radius."""

    pos: np.ndarray
    lo: tuple
    hi: tuple
    cell_size: float
    radius: float
    name: str = ""

    @property
    def dim(self) -> int:
        return int(self.pos.shape[1])

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def lattice(dim: int, n: int, dx: float, jitter: float = 0.1, seed: int = 0,
            radius_factor: float = 2.4, name: str = "") -> ParticleSet:
    """n^dim sites at (i + 1/2) dx in [0, n dx]^dim, each moved by U(-jitter dx, +jitter dx)
    per component. Particle index = ix + n (iy + n iz): x varies fastest.
    Search radius = cell size = radius_factor * dx (2h with h = 1.2 dx)."""
    axes = (np.arange(n, dtype=np.float64) + 0.5) * dx
    grids = np.meshgrid(*([axes] * dim), indexing="ij")
    # indexing="ij" makes the first axis slowest; reverse so x is fastest
    pos = np.stack([g.reshape(-1) for g in grids[::-1]], axis=1)
    pos = np.ascontiguousarray(pos)
    if jitter:
        rng = np.random.default_rng(seed)
        pos += rng.uniform(-jitter * dx, jitter * dx, size=pos.shape)
    L = n * dx
    r = radius_factor * dx
    return ParticleSet(pos, (0.0,) * dim, (L,) * dim, r, r, name or f"lattice{dim}d_n{n}")


def uniform(dim: int, npart: int, seed: int = 0, radius_factor: float = 2.4,
            box: float = 1.0, name: str = "") -> ParticleSet:
    """npart uniform points in [0, box]^dim; ds = box (1/N)^(1/d); radius = cell = 2.4 ds."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(npart, dim))
    ds = box * (1.0 / max(npart, 1)) ** (1.0 / dim)
    r = radius_factor * ds
    return ParticleSet(pos, (0.0,) * dim, (box,) * dim, r, r, name or f"uniform{dim}d_{npart}")


def clustered(npart: int, seed, dim: int = 3, nclusters: int = 8, background: float = 0.2,
              sigma=(0.02, 0.1), radius_factor: float = 2.4, name: str = "") -> ParticleSet:
    """A mixture: `background` of the points uniform in [0,1]^dim, the rest from `nclusters`
    equal-weight Gaussians with centres U[0,1]^dim and sigma ~ U(sigma). Draws that fall
    outside the box are drawn again. Radius = cell = 2.4 (1/N)^(1/d)."""
    rng = np.random.default_rng(seed)
    nbg = int(round(background * npart))
    ncl = npart - nbg
    centres = rng.uniform(0.0, 1.0, size=(nclusters, dim))
    sig = rng.uniform(sigma[0], sigma[1], size=nclusters)
    which = rng.integers(0, nclusters, size=ncl)
    pts = np.empty((ncl, dim))
    todo = np.arange(ncl)
    while todo.size:
        draw = centres[which[todo]] + rng.standard_normal((todo.size, dim)) * sig[which[todo], None]
        ok = np.all((draw >= 0.0) & (draw <= 1.0), axis=1)
        pts[todo[ok]] = draw[ok]
        todo = todo[~ok]
    pos = np.concatenate([rng.uniform(0.0, 1.0, size=(nbg, dim)), pts], axis=0)
    pos = pos[rng.permutation(npart)]
    r = radius_factor * (1.0 / npart) ** (1.0 / dim)
    return ParticleSet(np.ascontiguousarray(pos), (0.0,) * dim, (1.0,) * dim, r, r,
                       name or f"clustered{dim}d_{npart}")


def clustered_batch(nsets: int = 32, seed: int = 3, lo: float = 1e4, hi: float = 1e6,
                    dim: int = 3):
    """nsets clustered sets with sizes floor(exp(U(ln lo, ln hi))); seeds from
    SeedSequence(seed).spawn(nsets)."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(nsets)
    size_rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(size_rng.uniform(math.log(lo), math.log(hi), size=nsets))).astype(np.int64)
    return [clustered(int(s), kids[k], dim=dim, name=f"batch{k}_{int(s)}") for k, s in enumerate(sizes)]


def ring_pairs(npairs: int, radius: float, seed: int = 0, dim: int = 2, exps=(7, 9, 11, 13),
               box: float = 1.0):
    """Adversarial near-cutoff pairs: centres uniform in the box's inner part, partner at
    distance radius (1 + k 2^-m) for k in {-1, 0, +1} and m in `exps`, random direction.
    Mirrors the ring-of-particles accuracy test (Fig. 9, Table 1) at the cutoff."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(npairs):
        c = rng.uniform(0.25 * box, 0.75 * box, size=dim)
        m = exps[rng.integers(len(exps))]
        k = rng.integers(-1, 2)
        d = rng.standard_normal(dim)
        d /= np.linalg.norm(d)
        out.append(c)
        out.append(c + d * radius * (1.0 + k * 2.0 ** (-m)))
    pos = np.clip(np.array(out), 0.0, box)
    return ParticleSet(np.ascontiguousarray(pos), (0.0,) * dim, (box,) * dim, radius, radius,
                       f"ring{dim}d_{npairs}")


# Named workloads (the sizes quoted for this library's benchmarks and parity tests).
def c0():
    """2D 100x100 lattice, dx=0.01, jitter +-0.1dx, seed 0."""
    return lattice(2, 100, 0.01, 0.1, seed=0, name="lattice2d_100x100")


def c1():
    """2D 1000x1000 lattice, dx=1e-3 in [0,1]^2, jitter +-0.1dx, seed 1."""
    return lattice(2, 1000, 1e-3, 0.1, seed=1, name="lattice2d_1000x1000")


def c2():
    """3D 100x100x100 lattice, dx=0.01 in [0,1]^3, jitter +-0.1dx, seed 2."""
    return lattice(3, 100, 0.01, 0.1, seed=2, name="lattice3d_100x100x100")


def serving_sims(nsims: int = 64, seed: int = 4, lo: float = 1e3, hi: float = 2e6):
    """Serving mix: half 2D, half 3D lattices; sizes log-uniform in [lo, hi] snapped to n^d;
    dx = 1/n, radius 2.4 dx, jitter +-0.1dx."""
    rng = np.random.default_rng(seed)
    sims = []
    for s in range(nsims):
        dim = 2 if s < nsims // 2 else 3
        target = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        n = max(2, int(round(target ** (1.0 / dim))))
        sims.append(lattice(dim, n, 1.0 / n, 0.1, seed=seed * 1000 + s, name=f"sim{s}_{dim}d_{n}"))
    return sims


def step_displacement(ps: ParticleSet, step: int, seed: int, frac: float = 0.05) -> np.ndarray:
    """Per-step move U(-frac dx, +frac dx) per component, dx = radius / 2.4; walls reflect."""
    rng = np.random.default_rng([seed, step])
    dx = ps.radius / 2.4
    new = ps.pos + rng.uniform(-frac * dx, frac * dx, size=ps.pos.shape)
    lo = np.asarray(ps.lo)
    hi = np.asarray(ps.hi)
    new = np.where(new < lo, 2 * lo - new, new)
    new = np.where(new > hi, 2 * hi - new, new)
    return np.clip(new, lo, hi)


def reflected_displacement(pos: np.ndarray, lo, hi, amp: float, seed) -> np.ndarray:
    """A seeded displacement U(-amp, +amp) per component for the particles at `pos`, with the
    sign of a component flipped where pos + d (one binary64 addition, as the update applies
    it) would leave [lo, hi]; pos + d then stays inside the box while amp is well below the
    box size."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(-amp, amp, size=pos.shape)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    new = pos + d
    d = np.where((new < lo) | (new > hi), -d, d)
    new = pos + d
    assert np.all((new >= lo) & (new <= hi)), "displacement too large for the box"
    return np.ascontiguousarray(d)
