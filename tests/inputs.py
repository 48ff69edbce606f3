"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds none of the method's arithmetic: it only draws states and
parameters from numpy's seeded generator, so that both implementations can be
started from identical inputs.  The method's own random numbers (noise kicks,
random-sphere initial states) are NOT drawn here: each side implements
Philox4x32-10 from its published definition.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def unit_spins(n: int, seed: int) -> np.ndarray:
    """(3, n) float64 unit vectors, isotropic (normalised Gaussian triples)."""
    g = rng(seed).standard_normal((3, n))
    return g / np.linalg.norm(g, axis=0, keepdims=True)


def near_ordered_spins(n: int, seed: int, axis=(0.0, 0.0, 1.0), spread: float = 0.3) -> np.ndarray:
    """(3, n) unit vectors scattered around `axis` (a smooth-ish ferromagnetic state)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    g = rng(seed).standard_normal((3, n)) * spread + a[:, None]
    return g / np.linalg.norm(g, axis=0, keepdims=True)


def site_anisotropy(n: int, seed: int, mean: float = 0.1, std: float = 0.02):
    """Per-site D_i ~ N(mean, std^2) and isotropic random unit easy axes e_i (3, n)."""
    r = rng(seed)
    D = mean + std * r.standard_normal(n)
    e = r.standard_normal((3, n))
    e /= np.linalg.norm(e, axis=0, keepdims=True)
    return D, e


def batch_replicas(seed: int = 0, n_per_size: int = 32, sizes=(24, 48, 64)):
    """Replica table of the uneven batched workload: n_per_size replicas of each
    cubic size, T uniform in [0.3, 2.0], lambda log-uniform in [0.005, 0.05],
    one seed per replica."""
    r = rng(seed)
    reps = []
    idx = 0
    for L in sizes:
        for _ in range(n_per_size):
            T = 0.3 + 1.7 * r.random()
            lam = 0.005 * 10.0 ** r.random()
            reps.append({"L": (L, L, L), "T": float(T), "lam": float(lam),
                         "seed": int(1000 + idx), "replica": idx})
            idx += 1
    return reps
