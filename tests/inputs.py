"""Seeded synthetic inputs shared by the oracle side and the HIP side of the
tests.  This module holds none of the method's arithmetic: it only draws
arrays of given shapes from numpy's PCG64 generator.
"""
import numpy as np


def perturbed_populations(base, n_sites, rel, seed):
    """Populations base[i] * (1 + rel * z_is), z standard normal; shape (q, n_sites)."""
    rng = np.random.default_rng(seed)
    base = np.asarray(base, dtype=np.float64)
    z = rng.standard_normal((base.size, n_sites))
    return np.ascontiguousarray(base[:, None] * (1.0 + rel * z))


def random_field(n_sites, scale, seed, offset=0.0):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(offset + scale * rng.standard_normal(n_sites))
