"""Seeded synthetic inputs: density fields and random draws.

This module holds the input recipes only and none of the method's arithmetic, so that the
GPU library and the FP64 oracle can be fed the very same arrays. Arrays are indexed
[y][x] (2D) or [z][y][x] (3D), x fastest, and flattened in that order.
"""
from __future__ import annotations

import numpy as np


def droplet(dims, radius, n_in, n_out, width=3.0, center=None, noise=0.0, seed=0):
    """Circular (spherical) droplet with a tanh profile:
    n = n_out + (n_in - n_out) * (1 - tanh((r - R)/width)) / 2, r measured from ``center``
    (default: the site (L/2, L/2[, L/2]), 0-based). ``noise`` adds U(-noise, noise) from
    ``numpy.random.default_rng(seed)`` after the profile. Swap n_in/n_out for a bubble.
    """
    dims = tuple(int(v) for v in dims)
    if center is None:
        center = tuple(v // 2 for v in dims)
    grids = np.meshgrid(*[np.arange(v, dtype=np.float64) for v in reversed(dims)], indexing="ij")
    # grids are in [z][y][x] order; center is (x, y[, z])
    r2 = np.zeros(grids[0].shape)
    for g, c in zip(reversed(grids), center):
        r2 += (g - c) ** 2
    r = np.sqrt(r2)
    n = n_out + (n_in - n_out) * 0.5 * (1.0 - np.tanh((r - radius) / width))
    if noise:
        n = n + np.random.default_rng(seed).uniform(-noise, noise, n.shape)
    return np.ascontiguousarray(n.reshape(-1))


def uniform(dims, low, high, seed):
    """n ~ U(low, high) per site (spinodal-decomposition start)."""
    size = int(np.prod(dims))
    return np.random.default_rng(seed).uniform(low, high, size)


def around(dims, mean, amplitude, seed):
    """n = mean + U(-amplitude, amplitude) per site."""
    size = int(np.prod(dims))
    return mean + np.random.default_rng(seed).uniform(-amplitude, amplitude, size)


def slab(nx, n_in, n_out, half_width, width=3.0, ny=1):
    """Flat liquid slab centred in x (two interfaces), uniform along y: shape [ny][nx]."""
    x = np.arange(nx, dtype=np.float64)
    c = nx / 2.0
    prof = n_out + (n_in - n_out) * 0.5 * (np.tanh((x - (c - half_width)) / width)
                                             - np.tanh((x - (c + half_width)) / width))
    return np.ascontiguousarray(np.tile(prof, (ny, 1)).reshape(-1))


def knob_draws(seed, count, low, high):
    """``count`` values U(low, high) from ``numpy.random.default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(low, high, count)


def log_radii(count, rmin, rmax):
    """Radii spaced log-uniformly: R_k = rmin * (rmax/rmin)^(k/(count-1))."""
    k = np.arange(count, dtype=np.float64)
    return rmin * (rmax / rmin) ** (k / (count - 1))
