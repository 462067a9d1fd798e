"""Seeded synthetic inputs for the direct-summation N-body path.

This module is shared by the GPU library's tests/benchmark and by the CPU
oracle's tests; it holds no force, integrator or error arithmetic, only the
construction of initial conditions.  Every generator draws uniforms from
numpy's PCG64 stream and shapes them by inverse transforms written here, so a
seed fixes every array bit for bit.

Units: G = 1, total mass of a cluster = 1 (Henon/virial units for Plummer).

Generators
  plummer(n, seed)                Plummer sphere (Aarseth, Henon & Wielen 1974)
  cluster_batch(seed, n_clusters) many independent Plummer clusters, N log-uniform
  hernquist_merger(seed, ...)     11 Hernquist galaxies, a point mass in each,
                                  the i-set of stars near the point masses
"""
from dataclasses import dataclass

import numpy as np

__all__ = ["Particles", "plummer", "cluster_batch", "ClusterBatch", "hernquist_merger",
           "Merger", "plummer_eps2_c1", "PLUMMER_R_CUT"]

PLUMMER_R_CUT = 10.0  # radii drawn beyond this (Plummer scale units) are redrawn


@dataclass
class Particles:
    pos: np.ndarray   # (N,3) float64
    vel: np.ndarray   # (N,3) float64
    mass: np.ndarray  # (N,)  float64


def _rng(seed, *sub):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), *map(int, sub)])))


def _isotropic(rng, n):
    """Unit vectors uniform on the sphere: z uniform in [-1,1], azimuth uniform."""
    u = rng.random((n, 2))
    z = 1.0 - 2.0 * u[:, 0]
    phi = 2.0 * np.pi * u[:, 1]
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=1)


def plummer(n: int, seed: int) -> Particles:
    """Plummer sphere of n equal masses summing to 1, in Henon units (E ~ -1/4).

    Radii: r = (X^{-2/3} - 1)^{-1/2} with X uniform, redrawn when r > 10;
    speeds: v = q sqrt(2) (1 + r^2)^{-1/4} with q drawn by von Neumann
    rejection on g(q) = q^2 (1 - q^2)^{7/2} (envelope 0.1); isotropic
    directions; lengths scaled by 3 pi/16 and speeds by sqrt(16/(3 pi)); the
    centre of mass is moved to rest at the origin.  No exact virial rescaling.
    """
    if n < 1:
        raise ValueError("n >= 1")
    rng = _rng(seed, 0)
    r = np.empty(n)
    filled = 0
    while filled < n:
        x = rng.random(n - filled)
        with np.errstate(divide="ignore"):
            cand = 1.0 / np.sqrt(np.power(x, -2.0 / 3.0) - 1.0)
        cand = cand[np.isfinite(cand) & (cand <= PLUMMER_R_CUT) & (x > 0)]
        r[filled:filled + cand.size] = cand
        filled += cand.size
    pos = r[:, None] * _isotropic(rng, n)
    q = np.empty(n)
    filled = 0
    while filled < n:
        m = n - filled
        u = rng.random((m, 2))
        qq, yy = u[:, 0], 0.1 * u[:, 1]
        ok = qq[yy < qq * qq * np.power(1.0 - qq * qq, 3.5)]
        q[filled:filled + ok.size] = ok
        filled += ok.size
    speed = q * np.sqrt(2.0) * np.power(1.0 + r * r, -0.25)
    vel = speed[:, None] * _isotropic(rng, n)
    pos *= 3.0 * np.pi / 16.0
    vel *= np.sqrt(16.0 / (3.0 * np.pi))
    mass = np.full(n, 1.0 / n)
    pos -= (mass[:, None] * pos).sum(0) / mass.sum()
    vel -= (mass[:, None] * vel).sum(0) / mass.sum()
    return Particles(np.ascontiguousarray(pos), np.ascontiguousarray(vel), mass)


def plummer_eps2_c1():
    """Softening of the small Plummer case: eps = 0.01."""
    return 1e-4


@dataclass
class ClusterBatch:
    offsets: np.ndarray  # (C+1,) int64, cluster c owns rows offsets[c]:offsets[c+1]
    sizes: np.ndarray    # (C,) int64
    eps2: np.ndarray     # (C,) float64
    pos: np.ndarray
    vel: np.ndarray
    mass: np.ndarray


def cluster_batch(seed: int = 4, n_clusters: int = 128, n_min: int = 128, n_max: int = 16384) -> ClusterBatch:
    """Independent Plummer clusters, N_c = min(n_max, floor(n_min (n_max/n_min)^U)).

    U uniform from the batch stream; cluster c is plummer(N_c, seed derived
    from (seed, c)); each cluster has mass 1 and eps_c = 0.05 N_c^{-1/3}."""
    rng = _rng(seed, 1)
    u = rng.random(n_clusters)
    sizes = np.minimum(n_max, np.floor(n_min * np.power(n_max / n_min, u))).astype(np.int64)
    offsets = np.zeros(n_clusters + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    pos = np.empty((offsets[-1], 3)); vel = np.empty((offsets[-1], 3)); mass = np.empty(offsets[-1])
    for c in range(n_clusters):
        p = plummer(int(sizes[c]), seed * 1000003 + c)
        sl = slice(offsets[c], offsets[c + 1])
        pos[sl], vel[sl], mass[sl] = p.pos, p.vel, p.mass
    eps2 = (0.05 * np.power(sizes.astype(np.float64), -1.0 / 3.0)) ** 2
    return ClusterBatch(offsets, sizes, eps2, pos, vel, mass)


@dataclass
class Merger:
    pos: np.ndarray
    vel: np.ndarray
    mass: np.ndarray
    eps2: float
    bh_index: np.ndarray   # (G,) row of each point mass
    active: np.ndarray     # i-set, ascending int32
    centres: np.ndarray    # (G,3)


def hernquist_merger(seed: int = 5, n_gal: int = 11, n_star: int = 1 << 17,
                     bh_frac: float = 1e-3, r_place: float = 20.0, r_sel: float = 0.05) -> Merger:
    """Galaxies of unit mass and scale radius 1 with a central point mass.

    Stars: Hernquist radii r = sqrt(X)/(1 - sqrt(X)) with X uniform in
    [0, (10/11)^2) (cut at r = 10), isotropic directions, isotropic Gaussian
    velocities of 1-D dispersion v_c(r)/sqrt(3), v_c = sqrt(r)/(1 + r); the
    star centre of mass is moved onto the galaxy centre.  Point mass
    bh_frac at the centre.  Galaxy centres uniform on the sphere of radius
    r_place, moving radially inwards at sqrt(2 n_gal / r_place).  The
    softening is 0.05 n_star^{-1/3}.  The i-set is the point masses plus
    every star with |x - x_bh| < r_sel for some point mass (distance in
    double precision).  Rows: galaxy g's stars, then its point mass."""
    rows = n_gal * (n_star + 1)
    pos = np.empty((rows, 3)); vel = np.empty((rows, 3)); mass = np.empty(rows)
    rng0 = _rng(seed, 2)
    centres = r_place * _isotropic(rng0, n_gal)
    v_in = np.sqrt(2.0 * n_gal / r_place)
    bulk = -v_in * centres / r_place
    bh_index = np.zeros(n_gal, dtype=np.int64)
    for g in range(n_gal):
        rng = _rng(seed, 3, g)
        x = rng.random(n_star) * (10.0 / 11.0) ** 2
        sx = np.sqrt(x)
        r = sx / (1.0 - sx)
        p = r[:, None] * _isotropic(rng, n_star)
        sig = np.sqrt(r) / (1.0 + r) / np.sqrt(3.0)
        g3 = rng.standard_normal((n_star, 3))
        v = sig[:, None] * g3
        p -= p.mean(0)
        v -= v.mean(0)
        base = g * (n_star + 1)
        pos[base:base + n_star] = p + centres[g]
        vel[base:base + n_star] = v + bulk[g]
        mass[base:base + n_star] = (1.0 - bh_frac) / n_star
        pos[base + n_star] = centres[g]
        vel[base + n_star] = bulk[g]
        mass[base + n_star] = bh_frac
        bh_index[g] = base + n_star
    sel = np.zeros(rows, dtype=bool)
    sel[bh_index] = True
    for g in range(n_gal):
        d = pos - pos[bh_index[g]]
        sel |= np.sqrt((d * d).sum(1)) < r_sel
    active = np.nonzero(sel)[0].astype(np.int32)
    eps = 0.05 * n_star ** (-1.0 / 3.0)
    return Merger(pos, vel, mass, eps * eps, bh_index, active, centres)
