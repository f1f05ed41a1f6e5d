"""Seeded probes for comparing large fields without storing them.

Pure input description: which entries of a field are sampled, and the
Gaussian sketch vectors a field is projected on.  No solver arithmetic.

For a difference d of two fields and g with independent N(0, 1) entries,
E[(g . d)^2] = |d|^2, so the mean of (g_k . d)^2 over K independent vectors
estimates |d|^2 from K numbers per field (chi-square with K degrees of
freedom: for K = 16 the estimate of |d| is above 0.6 |d| with probability
0.99).
"""
from __future__ import annotations

import numpy as np


def sample_edges(candidates, step, m, seed):
    """m distinct entries of `candidates` (sorted), drawn for one step from
    default_rng((seed, step))."""
    rng = np.random.default_rng((seed, step))
    pick = rng.choice(len(candidates), m, replace=False)
    return np.sort(np.asarray(candidates)[pick])


def sketch_vectors(n, K, seed):
    """[K, n] float64 standard normal entries from default_rng(seed)."""
    return np.random.default_rng(seed).standard_normal((K, n))
