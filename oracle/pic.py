"""Oracle, part 3: the particle steps around the field solve (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain, slow on purpose:
every search is brute force over all tetrahedra (optionally narrowed by a
bounding-box test that cannot drop a tetrahedron that matters).

Sec. II-A: particles are delta shapes; their charge is measured by the
0-form (vertex hat functions lam_k) and their current by the 1-form (the
Whitney edge functions W_ij = lam_i g_j - lam_j g_i).  The time integral of
the current over a step is what reaches the field solve, so that the
discrete continuity equation, and with it the discrete Gauss law, holds
exactly.  For a particle of charge q moving on the straight path a -> b in
one step, the step-averaged edge current is

    J_e = (q / dt) * int_a^b W_e . dl.

The fields at a particle are the Whitney interpolants: E = sum_e e_e W_e
(edge 1-form), B = the face 2-form, which inside one tetrahedron is the
constant vector sum_e b_e curl W_e with curl W_ij = 2 g_i x g_j; Faraday's
law moves B by a multiple of curl E in every tetrahedron.

Newton's equations are advanced with the Adams-Bashforth scheme (Sec. II-A
names it; the order is not given): two steps here, on the first-order
system x' = v, v' = (q/m)(E + v x B), with one forward-Euler start step.
"""
from __future__ import annotations

import numpy as np

from .fem import LOCAL_EDGES, barycentric_gradients, canonical_edges, sort_tets


class TetMesh:
    """Sorted tetrahedra, their barycentric gradients and canonical edges."""

    def __init__(self, coords, tets):
        self.coords = np.asarray(coords, dtype=np.float64)
        self.st = sort_tets(tets)                        # [n_t, 4] ascending
        self.g, self.vol = barycentric_gradients(self.coords, tets)
        self.edges, self.tet_edges = canonical_edges(tets)
        self.n_e = len(self.edges)
        self.x0 = self.coords[self.st[:, 0]]             # lam = e_0 at vertex 0
        x = self.coords[self.st]
        self.lo = x.min(axis=1)                          # bounding boxes
        self.hi = x.max(axis=1)

    def lam(self, x, tets=None):
        """Barycentric coordinates [len(tets), 4] of point x in each tet:
        lam_k(x) = delta_k0 + g_k . (x - x_0)."""
        t = np.arange(len(self.st)) if tets is None else tets
        L = np.einsum("tkd,td->tk", self.g[t], x[None, :] - self.x0[t])
        L[:, 0] += 1.0
        return L

    def candidates(self, lo, hi, pad=1e-12):
        """Tets whose bounding box meets the box [lo, hi]."""
        m = np.all(self.lo <= hi + pad, axis=1) & np.all(self.hi >= lo - pad, axis=1)
        return np.flatnonzero(m)


def locate(mesh, x, tol=1e-12):
    """Containing tetrahedron of each point (the one whose smallest
    barycentric coordinate is largest); -1 outside the mesh."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    out = np.full(len(x), -1, dtype=np.int64)
    for p in range(len(x)):
        c = mesh.candidates(x[p], x[p])
        if len(c) == 0:
            continue
        m = mesh.lam(x[p], c).min(axis=1)
        k = int(np.argmax(m))
        if m[k] >= -tol:
            out[p] = c[k]
    return out


def whitney_field(mesh, e, cells, x):
    """E(x) = sum over the 6 edges of the cell of e_edge W_edge(x), [n, 3]."""
    x = np.atleast_2d(x)
    E = np.zeros((len(x), 3))
    for p in range(len(x)):
        t = cells[p]
        lam = mesh.lam(x[p], np.array([t]))[0]
        g = mesh.g[t]
        for a, (i, j) in enumerate(LOCAL_EDGES):
            E[p] += e[mesh.tet_edges[t, a]] * (lam[i] * g[j] - lam[j] * g[i])
    return E


def tet_curl(mesh, e):
    """Per-tetrahedron curl of the edge field: sum_e e_e 2 g_i x g_j, [n_t, 3]."""
    out = np.zeros((len(mesh.st), 3))
    for a, (i, j) in enumerate(LOCAL_EDGES):
        out += e[mesh.tet_edges[:, a]][:, None] * 2.0 * np.cross(mesh.g[:, i], mesh.g[:, j])
    return out


def faraday(mesh, e, B, alpha):
    """B + alpha * curl(E) in every tetrahedron (alpha = -dt for one step)."""
    return np.asarray(B, dtype=np.float64) + alpha * tet_curl(mesh, e)


def path_pieces(mesh, a, b, tol=1e-12):
    """Split the straight path a -> b where it crosses the plane of any face
    of any (candidate) tetrahedron; each piece lies in one tetrahedron, the
    one that contains its midpoint most deeply.  Returns [(s0, s1, t)]."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = mesh.candidates(np.minimum(a, b), np.maximum(a, b))
    La, Lb = mesh.lam(a, c), mesh.lam(b, c)
    den = La - Lb
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(den != 0.0, La / den, np.nan)
    s = s[np.isfinite(s)]
    s = np.unique(np.concatenate([[0.0, 1.0], s[(s > 0.0) & (s < 1.0)]]))
    out = []
    for s0, s1 in zip(s[:-1], s[1:]):
        if s1 <= s0:
            continue
        sm = 0.5 * (s0 + s1)
        Lm = (1.0 - sm) * La + sm * Lb
        m = Lm.min(axis=1)
        k = int(np.argmax(m))
        if m[k] < -tol:
            raise ValueError("path leaves the mesh")
        out.append((s0, s1, int(c[k])))
    return out


def deposit(mesh, a, b, q, dt):
    """Edge currents J [n_e] of straight paths a[p] -> b[p] with charges q[p].

    Inside one tetrahedron lam is linear along the piece, so
    int W_ij . dl = avg(lam_i) g_j . dr - avg(lam_j) g_i . dr exactly.  (On a
    straight piece the integrand lam_i dlam_j - lam_j dlam_i is constant,
    so lam at any point of the piece gives the same value.)"""
    a = np.atleast_2d(np.asarray(a, dtype=np.float64))
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    q = np.broadcast_to(np.asarray(q, dtype=np.float64), (len(a),))
    J = np.zeros(mesh.n_e)
    for p in range(len(a)):
        for s0, s1, t in path_pieces(mesh, a[p], b[p]):
            p0 = a[p] + s0 * (b[p] - a[p])
            p1 = a[p] + s1 * (b[p] - a[p])
            l0 = mesh.lam(p0, np.array([t]))[0]
            l1 = mesh.lam(p1, np.array([t]))[0]
            lavg = 0.5 * (l0 + l1)
            gdr = mesh.g[t] @ (p1 - p0)                   # g_k . dr = change of lam_k
            for k, (i, j) in enumerate(LOCAL_EDGES):
                J[mesh.tet_edges[t, k]] += q[p] / dt * (lavg[i] * gdr[j] - lavg[j] * gdr[i])
    return J


def lorentz(qm, E, B, v):
    """Acceleration (q/m)(E + v x B) of each particle, [n, 3]."""
    return np.asarray(qm)[:, None] * (E + np.cross(v, B))


def push_ab2(x, v, acc, hist_v, hist_a, dt, first):
    """One Adams-Bashforth step of x' = v, v' = acc.

    first: forward Euler (no history yet).  Otherwise
      x+ = x + dt (3/2 v - 1/2 v_prev),  v+ = v + dt (3/2 acc - 1/2 acc_prev).
    Returns (x+, v+, new history (v, acc))."""
    if first:
        xn = x + dt * v
        vn = v + dt * acc
    else:
        xn = x + dt * (1.5 * v - 0.5 * hist_v)
        vn = v + dt * (1.5 * acc - 0.5 * hist_a)
    return xn, vn, v.copy(), acc.copy()
