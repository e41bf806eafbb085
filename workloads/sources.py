"""Right-hand-side source functions and random vectors for the workloads.

A source is a plain function of the physical position; how it is integrated
against the finite element basis is the consumer's business.
"""

from __future__ import annotations

import numpy as np

from .meshes import CONFIGS, _seed_base

BUMP_WIDTH = 0.1


def gaussian_bumps(x: np.ndarray, centres: np.ndarray, width: float = BUMP_WIDTH) -> np.ndarray:
    """f(x) = sum_g exp(-|x - c_g|^2 / (2 width^2)) for points x [..., dim]."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape[:-1], dtype=np.float64)
    for c in centres:
        d2 = np.sum((x - c) ** 2, axis=-1)
        out += np.exp(-d2 / (2.0 * width * width))
    return out


def bump_centres_cube(dim: int, rng: np.random.Generator, count: int = 8) -> np.ndarray:
    """Bump centres uniform in [0.1, 0.9]^dim."""
    return rng.uniform(0.1, 0.9, size=(count, dim))


def bump_centres_ball(dim: int, rng: np.random.Generator, count: int = 8, radius: float = 0.8) -> np.ndarray:
    """Bump centres uniform in the ball of the given radius (rejection sampling)."""
    out = []
    while len(out) < count:
        p = rng.uniform(-radius, radius, size=dim)
        if np.dot(p, p) < radius * radius:
            out.append(p)
    return np.array(out)


def config_source(cfg, rhs_id: int = 0):
    """The source function of a workload: a callable x [..., dim] -> f [...].

    Bump centres are drawn with ``numpy.random.default_rng(2000 * cfg_seed + rhs_id)``.
    """
    c = CONFIGS[cfg]
    kind = c["source"]
    if kind == "one":
        return lambda x: np.ones(np.asarray(x).shape[:-1], dtype=np.float64)
    if kind == "gravity":
        # vector body load (0, 0, -1): x [..., 3] -> f [..., 3]
        def gravity(x):
            x = np.asarray(x, dtype=np.float64)
            f = np.zeros(x.shape[:-1] + (3,))
            f[..., 2] = -1.0
            return f
        return gravity
    rng = np.random.default_rng(2000 * _seed_base(cfg) + rhs_id)
    if kind == "bumps":
        cen = bump_centres_cube(c["dim"], rng)
    elif kind == "bumps_ball":
        cen = bump_centres_ball(c["dim"], rng)
    else:
        raise ValueError(kind)
    return lambda x: gaussian_bumps(x, cen)


def random_vector(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Seeded uniform float64 vector (used for operator inputs and Lanczos start vectors)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


def random_load(rhs_id: int, count: int = 4, width: float = 0.3):
    """Smooth random vector body load on the beam: per component a sum of
    `count` Gaussian bumps of the given width with random centres in the beam
    and random signed amplitudes, from numpy.random.default_rng(3000 + rhs_id)."""
    rng = np.random.default_rng(3000 + rhs_id)
    cen = rng.uniform((0.0, 0.0, 0.0), (5.0, 1.0, 1.0), size=(3, count, 3))
    amp = rng.uniform(-1.0, 1.0, size=(3, count))

    def load(x):
        x = np.asarray(x, dtype=np.float64)
        f = np.zeros(x.shape[:-1] + (3,))
        for c in range(3):
            for g in range(count):
                d2 = np.sum((x - cen[c, g]) ** 2, axis=-1)
                f[..., c] += amp[c, g] * np.exp(-d2 / (2.0 * width * width))
        return f
    return load
