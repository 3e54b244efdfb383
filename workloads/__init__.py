"""Seeded synthetic particle sets for the short-range PP gravity path.

This module only draws inputs: positions, masses and per-box parameters.
It holds none of the force, key, leaf or pair arithmetic, so both the CPU
oracle and the HIP library may be fed from it without sharing any code.

The workloads stand in for the clustered cosmological particle sets the
paper's PP kernel runs on (sec. 5: 128^3 particles in a 100 Mpc/h box
evolved from z=49 to 0); the paper's own initial conditions are not used.
Each set is a mixture of

* a uniform part, x ~ U[0, L)^3, and
* Plummer spheres whose particle counts follow dN/dM ~ M^-1.9 on
  [64, M_max] (M_max solved so the expected mean is N_cl / n_sph), scale
  radii a = 0.05 (M / nbar)^(1/3), radii drawn from the Plummer cumulative
  mass profile truncated at 10 a, isotropic directions, wrapped mod L.

All particles have mass 1/N and the gravitational constant is 1.
Split parameters follow the PM-Tree convention of sec. 3.1: the PM cell is
L / N_g, the split scale is r_s = 1.25 cells, the cut is 4.5 r_s and the
Plummer softening is 0.02 cells.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 180209824
M_MIN = 64.0
SLOPE = 1.9


@dataclasses.dataclass(frozen=True)
class BoxParams:
    """Per-box parameters of the short-range sum (lengths in Mpc/h)."""

    L: float
    rs: float
    rcut: float
    eps: float
    G: float = 1.0
    leaf_max: int = 32
    key_bits: int = 21

    @staticmethod
    def from_mesh(L: float, n_mesh: int, G: float = 1.0, leaf_max: int = 32,
                  key_bits: int = 21) -> "BoxParams":
        cell = L / n_mesh
        rs = 1.25 * cell
        return BoxParams(L=L, rs=rs, rcut=4.5 * rs, eps=0.02 * cell, G=G,
                         leaf_max=leaf_max, key_bits=key_bits)


@dataclasses.dataclass
class Box:
    """One periodic box: SoA float64 positions [3, n], float32 masses [n]."""

    pos: np.ndarray
    mass: np.ndarray
    params: BoxParams
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])


def rng_for(cfg: int, box: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 100 * cfg + box))


def uniform(rng: np.random.Generator, n: int, L: float) -> np.ndarray:
    """n points uniform in [0, L)^3, SoA float64 [3, n]."""
    return rng.random((3, n)) * L


def _powerlaw_mean(m_max: float) -> float:
    a = 1.0 - SLOPE           # exponent of the cumulative count
    num = (m_max ** (a + 1) - M_MIN ** (a + 1)) / (a + 1)
    den = (m_max ** a - M_MIN ** a) / a
    return num / den


def _solve_m_max(mean: float) -> float:
    if mean <= M_MIN * 1.0001:
        return M_MIN * 1.0002
    lo, hi = M_MIN * 1.0001, 1e12
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if _powerlaw_mean(mid) < mean:
            lo = mid
        else:
            hi = mid
    return math.sqrt(lo * hi)


def sphere_counts(rng: np.random.Generator, n_cl: int, n_sph: int) -> np.ndarray:
    """Particle counts of n_sph spheres, dN/dM ~ M^-1.9, summing to n_cl."""
    if n_sph <= 0 or n_cl <= 0:
        return np.zeros(0, dtype=np.int64)
    m_max = _solve_m_max(n_cl / n_sph)
    a = 1.0 - SLOPE
    u = rng.random(n_sph)
    lo, hi = M_MIN ** a, m_max ** a
    m = (lo + u * (hi - lo)) ** (1.0 / a)
    share = m / m.sum() * n_cl
    counts = np.floor(share).astype(np.int64)
    counts = np.maximum(counts, 1)
    # largest remainder to hit n_cl exactly (min 1 each)
    diff = n_cl - int(counts.sum())
    if diff > 0:
        order = np.argsort(-(share - np.floor(share)), kind="stable")
        counts[order[:diff]] += 1
    while diff < 0:
        order = np.argsort(-counts, kind="stable")
        take = min(-diff, int(np.count_nonzero(counts > 1)))
        counts[order[:take]] -= 1
        diff += take
    assert int(counts.sum()) == n_cl
    return counts


def plummer_spheres(rng: np.random.Generator, n_cl: int, n_sph: int, L: float,
                    nbar: float) -> np.ndarray:
    """n_cl points in n_sph Plummer spheres, SoA float64 [3, n_cl] in [0, L)."""
    counts = sphere_counts(rng, n_cl, n_sph)
    if counts.size == 0:
        return np.zeros((3, 0))
    centres = rng.random((3, counts.size)) * L
    scale = 0.05 * (counts / nbar) ** (1.0 / 3.0)
    owner = np.repeat(np.arange(counts.size), counts)
    umax = (100.0 / 101.0) ** 1.5
    u = rng.random(n_cl) * umax
    u = np.where(u <= 0.0, umax * 1e-12, u)       # (0, umax]
    r = scale[owner] / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    v = rng.standard_normal((3, n_cl))
    v /= np.linalg.norm(v, axis=0, keepdims=True)
    pos = centres[:, owner] + r * v
    return np.mod(pos, L)


def mixture(rng: np.random.Generator, n: int, L: float, frac_cl: float,
            n_sph: int) -> np.ndarray:
    n_cl = int(round(n * frac_cl))
    n_un = n - n_cl
    nbar = n / L ** 3
    parts = [uniform(rng, n_un, L)]
    if n_cl:
        parts.append(plummer_spheres(rng, n_cl, n_sph, L, nbar))
    pos = np.concatenate(parts, axis=1)
    # shuffle so that input order carries no spatial information
    perm = rng.permutation(n)
    pos = np.ascontiguousarray(pos[:, perm])
    # np.mod can return L itself for tiny negatives; keep [0, L)
    pos[pos >= L] -= L
    return pos


def equal_masses(n: int) -> np.ndarray:
    return np.full(n, 1.0 / max(n, 1), dtype=np.float32)


# The five workloads: (n, L, N_g, clustered fraction, spheres)
CONFIGS = {
    1: dict(n=32 ** 3, L=100.0, n_mesh=32, frac=0.0, n_sph=0,
            name="plain-32k-uniform-L100"),
    2: dict(n=128 ** 3, L=200.0, n_mesh=128, frac=0.5, n_sph=2000,
            name="plain-2M-clustered-L200"),
    3: dict(n=256 ** 3, L=400.0, n_mesh=256, frac=0.5, n_sph=8000,
            name="precision-16.8M-clustered-L400"),
    5: dict(n=512 ** 3, L=1000.0, n_mesh=512, frac=0.6, n_sph=50000,
            name="large-134M-clustered-L1000"),
}


def make_config(cfg: int, n: int | None = None) -> Box:
    """Box for workload cfg (1, 2, 3 or 5); n overrides the particle count
    (the density and split parameters then follow from the same L and mesh)."""
    c = CONFIGS[cfg]
    nn = c["n"] if n is None else int(n)
    rng = rng_for(cfg)
    n_sph = c["n_sph"] if n is None else max(1, int(round(c["n_sph"] * nn / c["n"]))) if c["n_sph"] else 0
    pos = mixture(rng, nn, c["L"], c["frac"], n_sph)
    return Box(pos=pos, mass=equal_masses(nn),
               params=BoxParams.from_mesh(c["L"], c["n_mesh"]), name=c["name"])


def make_batch(n_boxes: int = 64, n_lo: int = 16 ** 3, n_hi: int = 96 ** 3,
               cfg: int = 4) -> list[Box]:
    """Independent periodic boxes of different size, length and clustering."""
    boxes = []
    for b in range(n_boxes):
        rng = rng_for(cfg, b)
        n = int(rng.integers(n_lo, n_hi + 1))
        L = float(rng.uniform(50.0, 300.0))
        frac = float(rng.uniform(0.0, 0.8))
        n_cl = int(round(n * frac))
        n_sph = max(1, int(round(n_cl / 512)))
        n_mesh = int(round(n ** (1.0 / 3.0)))
        pos = mixture(rng, n, L, frac, n_sph)
        boxes.append(Box(pos=pos, mass=equal_masses(n),
                         params=BoxParams.from_mesh(L, n_mesh),
                         name=f"batch-box{b}-n{n}-L{L:.1f}"))
    return boxes


def lattice(n_side: int, L: float) -> np.ndarray:
    """Perfect cubic lattice with n_side^3 points at cell centres."""
    g = (np.arange(n_side) + 0.5) * (L / n_side)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()]).astype(np.float64)
