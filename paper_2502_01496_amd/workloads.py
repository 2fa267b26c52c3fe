"""Seeded synthetic workloads for the gravity path.

This module only draws inputs (positions, masses, smoothing lengths, cotangents);
it holds none of the force method's arithmetic.  Both the HIP path's tests and
benchmark and the CPU oracle's tests take their inputs from here.

Workloads (all use numpy ``Generator(PCG64(seed))``):

* ``plummer``   -- Plummer sphere by inverse-CDF radii and isotropic directions,
                   equal masses, fixed softening length.
* ``polytrope_binary`` -- two n=1 polytropes (the neutron-star model of Sec. 6 of
                   the paper: equal-mass particles, uniform isotropic positions
                   stretch-mapped along the mass coordinate, zero velocity).
* ``clumpy_cube`` -- uniform cube plus Gaussian clumps with log-normal masses.
* ``knn_h``     -- per-particle h from the 58-neighbour estimate of Sec. 6
                   (mean neighbour number 4/3 pi (R_kern h_fact)^3 ~ 57.9 for the
                   M4 kernel with h_fact = 1.2): h_i = d_57(i) / R_kern, where
                   d_k is the distance to the k-th nearest other particle, so the
                   closed ball of radius R_kern h_i holds 58 particles with i.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

_CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      ".workload_cache")


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _unit_open(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform on (0, 1): exact zeros are redrawn."""
    u = rng.random(n)
    bad = u == 0.0
    while bad.any():
        u[bad] = rng.random(int(bad.sum()))
        bad = u == 0.0
    return u


def _directions(rng: np.random.Generator, n: int) -> np.ndarray:
    mu = 2.0 * rng.random(n) - 1.0
    phi = 2.0 * np.pi * rng.random(n)
    st = np.sqrt(1.0 - mu * mu)
    return np.stack([st * np.cos(phi), st * np.sin(phi), mu], axis=1)


def plummer(n: int, seed: int, a: float = 1.0, mass: float = 1.0, h: float = 0.01):
    """Plummer sphere, no truncation: r = a / sqrt(u^(-2/3) - 1)."""
    rng = _rng(seed)
    u = _unit_open(rng, n)
    r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    x = r[:, None] * _directions(rng, n)
    m = np.full(n, mass / n)
    hh = np.full(n, float(h))
    return np.ascontiguousarray(x), m, hh


def polytrope_radius(mass_fraction: np.ndarray) -> np.ndarray:
    """Invert F(r) = (sin(pi r) - pi r cos(pi r)) / pi, the enclosed-mass fraction
    of an n=1 polytrope of radius 1, by bisection to ~1e-15."""
    target = np.asarray(mass_fraction, dtype=np.float64)
    lo = np.zeros_like(target)
    hi = np.ones_like(target)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        f = (np.sin(np.pi * mid) - np.pi * mid * np.cos(np.pi * mid)) / np.pi
        below = f < target
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return 0.5 * (lo + hi)


def polytrope_star(n: int, rng: np.random.Generator) -> np.ndarray:
    """n particles of an n=1 polytrope (radius 1) centred at the origin."""
    ru = rng.random(n) ** (1.0 / 3.0)           # uniform ball
    dirs = _directions(rng, n)
    r = polytrope_radius(ru ** 3)               # stretch map along the mass coordinate
    return r[:, None] * dirs


def knn_h(x: np.ndarray, k_other: int = 57, r_kern: float = 2.0, workers: int = -1):
    from scipy.spatial import cKDTree

    tree = cKDTree(x)
    d, _ = tree.query(x, k=k_other + 1, workers=workers)
    return np.ascontiguousarray(d[:, k_other] / r_kern)


def _cached(tag: str, fn):
    """Cache (x, m, h) triples on disk under .workload_cache/ keyed by tag."""
    os.makedirs(_CACHE, exist_ok=True)
    key = hashlib.sha1(tag.encode()).hexdigest()[:16]
    path = os.path.join(_CACHE, f"{key}.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            return z["x"], z["m"], z["h"]
    x, m, h = fn()
    tmp = path + f".{os.getpid()}.tmp.npz"
    np.savez(tmp, x=x, m=m, h=h)
    os.replace(tmp, path)
    return x, m, h


def polytrope_binary(n_per_star: int, seed: int, separation: float = 4.0,
                     cache: bool = True):
    """Two n=1 polytropes (M = 1, R = 1 each) centred at (+-separation/2, 0, 0),
    equal particle masses 1/n_per_star, h from the 58-neighbour estimate over
    both stars."""

    def make():
        rng = _rng(seed)
        a = polytrope_star(n_per_star, rng)
        b = polytrope_star(n_per_star, rng)
        a[:, 0] -= 0.5 * separation
        b[:, 0] += 0.5 * separation
        x = np.ascontiguousarray(np.concatenate([a, b]))
        m = np.full(2 * n_per_star, 1.0 / n_per_star)
        return x, m, knn_h(x)

    if not cache:
        return make()
    return _cached(f"polytrope_binary:{n_per_star}:{seed}:{separation}", make)


def polytrope_single(n: int, seed: int, cache: bool = True):
    """One n=1 polytrope (M = 1, R = 1) of n equal-mass particles at the
    origin, h from the 58-neighbour estimate."""

    def make():
        rng = _rng(seed)
        x = np.ascontiguousarray(polytrope_star(n, rng))
        return x, np.full(n, 1.0 / n), knn_h(x)

    if not cache:
        return make()
    return _cached(f"polytrope_single:{n}:{seed}", make)


def clumpy_cube(n: int, seed: int, n_clumps: int = 64, sigma: float = 0.02,
                clump_mass: float = 0.3, mass_sigma: float = 0.5, cache: bool = True):
    """Uniform [0,1)^3 background plus n_clumps Gaussian clumps holding
    clump_mass of the unit total mass; masses log-normal (sigma mass_sigma)."""

    def make():
        rng = _rng(seed)
        nc = int(np.floor(0.3 * n))
        per = nc // n_clumps
        sizes = np.full(n_clumps, per)
        sizes[: nc - per * n_clumps] += 1
        centres = rng.random((n_clumps, 3))
        parts = [centres[k] + sigma * rng.standard_normal((sizes[k], 3)) for k in range(n_clumps)]
        clump = np.concatenate(parts)
        bg = rng.random((n - nc, 3))
        x = np.ascontiguousarray(np.concatenate([clump, bg]))
        w = np.exp(mass_sigma * rng.standard_normal(n))
        m = np.empty(n)
        m[:nc] = w[:nc] * (clump_mass / w[:nc].sum())
        m[nc:] = w[nc:] * ((1.0 - clump_mass) / w[nc:].sum())
        return x, m, knn_h(x)

    if not cache:
        return make()
    return _cached(f"clumpy_cube:{n}:{seed}:{n_clumps}:{sigma}:{clump_mass}:{mass_sigma}", make)


def cotangent(n: int, seed: int) -> np.ndarray:
    """Standard-normal cotangent for the accelerations (n x 3)."""
    return np.ascontiguousarray(_rng(seed).standard_normal((n, 3)))


# Named configurations: sizes of the paper-derived workloads.
def config(name: str):
    """Return (x, m, h, theta) for a named workload.

    plummer_4096        Plummer, N = 4096, h = 0.01 (theta = 0.5)
    binary_2x2^18       n=1 polytrope binary, 2 x 2^18, 58-neighbour h (theta = 0.5)
    clumpy_2^22         clumpy cube, 2^22, 58-neighbour h (theta = 0.5)
    plummer_2^20        Plummer, N = 2^20, h = 0.01 (theta = 0.5)
    binary_2x2^23       n=1 polytrope binary, 2 x 2^23 (theta = 0.5)
    """
    if name == "plummer_4096":
        return (*plummer(4096, 1), 0.5)
    if name == "binary_2x2^18":
        return (*polytrope_binary(1 << 18, 2), 0.5)
    if name == "clumpy_2^22":
        return (*clumpy_cube(1 << 22, 3), 0.5)
    if name == "plummer_2^20":
        return (*plummer(1 << 20, 4), 0.5)
    if name == "binary_2x2^23":
        return (*polytrope_binary(1 << 23, 5), 0.5)
    raise KeyError(name)
