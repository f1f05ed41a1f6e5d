"""Seeded particle-beam source currents for the 64^3 cavity workload.

Sec. II-A maps particles to the mesh with delta shapes: the current is a
1-form, and its time integral over a step makes the discrete continuity
equation (and so the discrete Gauss law) exact.  For a straight particle
path from a to b the step-averaged edge current is

    J_i^{n+1/2} = dt^-1 sum_p q_p int_{a_p}^{b_p} W_i . dl,

evaluated exactly by splitting the path at tetrahedron faces (hexahedron
planes and the Kuhn planes f_a = f_b of each hexahedron) and using, inside
one tetrahedron, int W_ij . dl = avg(lam_i) g_j.dr - avg(lam_j) g_i.dr
(lam is linear along the piece).  This generator is an input producer only:
the particle push is not part of the solve (the beam moves ballistically).

Beam: `particles` macro-particles per right-hand side from default_rng(seed+r):
radius 0.2 sqrt(U), angle 2 pi U about the axis (0.5, 0.5), z ~ U[0, 1),
v_x, v_y ~ N(0, vth^2), v_z = vz, charge (-1)^p q0.  A particle leaving
through z = 1 re-enters at z = 0 with the same (x, y, v); both points are on
the conducting wall, so the interior Gauss law stays exact.
"""
from __future__ import annotations

import numpy as np

from .mesh import PERMS, mesh_edges

_PERM_ARR = np.array(PERMS, dtype=np.int64)
_PERM_INDEX = {p: i for i, p in enumerate(PERMS)}
LOCAL_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


class BeamSampler:
    def __init__(self, n, particles, radius, vth, vz, q0, seed):
        rng = np.random.default_rng(seed)
        rad = radius * np.sqrt(rng.uniform(0.0, 1.0, particles))
        th = 2.0 * np.pi * rng.uniform(0.0, 1.0, particles)
        z = rng.uniform(0.0, 1.0, particles)
        vx = rng.normal(0.0, vth, particles)
        vy = rng.normal(0.0, vth, particles)
        self.x0 = np.stack([0.5 + rad * np.cos(th), 0.5 + rad * np.sin(th), z], axis=1)
        self.v = np.stack([vx, vy, np.full(particles, vz)], axis=1)
        self.q = np.where(np.arange(particles) % 2 == 0, q0, -q0)
        self.n = n

    def positions(self, t):
        p = self.x0 + self.v * t
        p[:, 2] = np.mod(p[:, 2], 1.0)
        return p

    def segments(self, t0, t1):
        """Straight pieces (a, b, q) of every path over [t0, t1], split at the
        z = 1 -> z = 0 re-entry."""
        a = self.x0 + self.v * t0
        b = self.x0 + self.v * t1
        wa = np.floor(a[:, 2])
        wb = np.floor(b[:, 2])
        a[:, 2] -= wa
        b[:, 2] -= wa
        cross = wb > wa
        # piece 1: a -> wall (z = 1); piece 2: (z = 0) -> b - 1
        s = np.where(cross, (1.0 - a[:, 2]) / np.where(cross, b[:, 2] - a[:, 2], 1.0), 1.0)
        w = a + (b - a) * s[:, None]
        w[cross, 2] = 1.0
        A = [a, np.where(cross[:, None], w - np.array([0, 0, 1.0]), 0.0)[cross]]
        B = [np.where(cross[:, None], w, b), (b - np.array([0, 0, 1.0]))[cross]]
        Q = [self.q, self.q[cross]]
        return np.concatenate(A), np.concatenate(B), np.concatenate(Q)


def _split(a, b, idx, cuts):
    """Pieces [s0, s1] of segments idx at parameters cuts [m, k] (nan = none)."""
    m = len(idx)
    S = np.concatenate([np.zeros((m, 1)), np.where(np.isnan(cuts), 1.0, cuts), np.ones((m, 1))], axis=1)
    S.sort(axis=1)
    s0 = S[:, :-1].ravel()
    s1 = S[:, 1:].ravel()
    rep = np.repeat(idx, S.shape[1] - 1)
    keep = s1 > s0
    return rep[keep], s0[keep], s1[keep]


def deposit(n, edge_key_sorted, nv1, a, b, q, dt, n_e):
    """Edge currents of straight paths a -> b (uniform n^3 Kuhn mesh of the
    unit cube, vertex id (i(n+1)+j)(n+1)+k).  Returns J [n_e]."""
    J = np.zeros(n_e)
    m = len(a)
    d = b - a
    # ---- hexahedron planes ----------------------------------------------------
    ca = np.minimum(np.floor(a * n), n - 1)
    cb = np.minimum(np.floor(b * n), n - 1)
    cuts = np.full((m, 3), np.nan)
    for ax in range(3):
        c = ca[:, ax] != cb[:, ax]
        k = np.maximum(ca[c, ax], cb[c, ax])
        cuts[c, ax] = (k / n - a[c, ax]) / d[c, ax]
    seg, s0, s1 = _split(a, b, np.arange(m), cuts)
    P0 = a[seg] + d[seg] * s0[:, None]
    P1 = a[seg] + d[seg] * s1[:, None]
    hx = np.clip(np.floor(0.5 * (P0 + P1) * n), 0, n - 1)
    F0 = np.clip(P0 * n - hx, 0.0, 1.0)
    F1 = np.clip(P1 * n - hx, 0.0, 1.0)
    # ---- Kuhn planes f_a = f_b inside the hexahedron -----------------------------
    cuts = np.full((len(seg), 3), np.nan)
    for c, (i, j) in enumerate(((0, 1), (0, 2), (1, 2))):
        d0 = F0[:, i] - F0[:, j]
        d1 = F1[:, i] - F1[:, j]
        x = d0 * d1 < 0
        cuts[x, c] = d0[x] / (d0[x] - d1[x])
    pc, u0, u1 = _split(F0, F1, np.arange(len(seg)), cuts)
    dF = F1[pc] - F0[pc]
    G0 = F0[pc] + dF * u0[:, None]
    G1 = F0[pc] + dF * u1[:, None]
    gd = G1 - G0
    mid = 0.5 * (G0 + G1)
    perm = np.argsort(-mid, axis=1, kind="stable")      # p0, p1, p2: descending f
    rows = np.arange(len(pc))

    def lam(G):
        f0, f1, f2 = G[rows, perm[:, 0]], G[rows, perm[:, 1]], G[rows, perm[:, 2]]
        return np.stack([1.0 - f0, f0 - f1, f1 - f2, f2], axis=1)

    lavg = 0.5 * (lam(G0) + lam(G1))
    e0, e1, e2 = gd[rows, perm[:, 0]], gd[rows, perm[:, 1]], gd[rows, perm[:, 2]]
    gdr = np.stack([-e0, e0 - e1, e1 - e2, e2], axis=1)    # g_k . dr (h cancels)
    # vertex ids of the tetrahedron walk v0 -> v0 + e_p0 -> ... -> v0 + (1,1,1)
    hv = hx[pc].astype(np.int64)
    stride = np.array([(n + 1) * (n + 1), n + 1, 1], dtype=np.int64)
    v = np.empty((len(pc), 4), dtype=np.int64)
    v[:, 0] = hv @ stride
    v[:, 1] = v[:, 0] + stride[perm[:, 0]]
    v[:, 2] = v[:, 1] + stride[perm[:, 1]]
    v[:, 3] = v[:, 2] + stride[perm[:, 2]]
    w = q[seg[pc]] / dt
    for (i, j) in LOCAL_EDGES:
        val = w * (lavg[:, i] * gdr[:, j] - lavg[:, j] * gdr[:, i])
        key = v[:, i] * nv1 + v[:, j]
        e = np.searchsorted(edge_key_sorted, key)
        J += np.bincount(e, weights=val, minlength=n_e)
    return J


def beam_source(coords, tets, edges, n, N, dt, nrhs, particles, radius, vth, vz, q0, seed,
                steps=None, chunk=250_000):
    """J_half [len(steps), nrhs, n_e] for the given step indices (default:
    0..N-1); boundary entries are zeroed."""
    from .mesh import boundary_edge_mask
    nv1 = len(coords)
    keys = edges[:, 0].astype(np.int64) * nv1 + edges[:, 1]
    bnd = boundary_edge_mask(coords, edges)
    steps = range(N) if steps is None else steps
    steps = list(steps)
    J = np.zeros((len(steps), nrhs, len(edges)))
    for r in range(nrhs):
        bs = BeamSampler(n, particles, radius, vth, vz, q0, seed + r)
        for si, st in enumerate(steps):
            a, b, q = bs.segments(st * dt, (st + 1) * dt)
            acc = np.zeros(len(edges))
            for c0 in range(0, len(a), chunk):
                acc += deposit(n, keys, nv1, a[c0:c0 + chunk], b[c0:c0 + chunk], q[c0:c0 + chunk], dt,
                               len(edges))
            acc[bnd] = 0.0
            J[si, r] = acc
    return J
