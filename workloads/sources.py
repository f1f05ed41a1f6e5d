"""Seeded source currents for the Newmark field update.

Each generator returns J_half with shape [N][nrhs][n_e] (float64): entry
[n][r][i] is the step-averaged, Galerkin-projected current J_i^{n+1/2} on
canonical edge i for right-hand side r.  Entries on boundary (PEC) edges are
set to zero (they carry no unknown).  The current before the first step,
J^{-1/2}, is zero.

The pulse is p(t) = exp(-(t - t0)^2 / (2 sigma^2)) sampled at t_{n+1/2}.
"""
from __future__ import annotations

import numpy as np


def pulse(N: int, dt: float, t0: float, sigma: float):
    t = (np.arange(N, dtype=np.float64) + 0.5) * dt
    return np.exp(-((t - t0) ** 2) / (2.0 * sigma ** 2))


def dense_random_source(n_e, interior_mask, N, dt, t0, sigma, seed, nrhs=1,
                        seed_stride=1):
    """J_i = a_i p(t), a ~ U[-1, 1] over all canonical edges (one draw of n_e
    numbers per right-hand side from default_rng(seed + r*seed_stride))."""
    p = pulse(N, dt, t0, sigma)
    J = np.zeros((N, nrhs, n_e))
    for r in range(nrhs):
        a = np.random.default_rng(seed + r * seed_stride).uniform(-1.0, 1.0, n_e)
        a[~interior_mask] = 0.0
        J[:, r, :] = p[:, None] * a[None, :]
    return J


def sparse_random_source(n_e, interior_mask, N, dt, t0, sigma, seed, count):
    """`count` distinct interior edges from default_rng(seed).choice, with
    amplitudes U[-1, 1] drawn next from the same generator; one RHS."""
    rng = np.random.default_rng(seed)
    interior = np.flatnonzero(interior_mask)
    pick = rng.choice(len(interior), count, replace=False)
    amp = rng.uniform(-1.0, 1.0, count)
    p = pulse(N, dt, t0, sigma)
    J = np.zeros((N, 1, n_e))
    J[:, 0, interior[pick]] = p[:, None] * amp[None, :]
    return J
