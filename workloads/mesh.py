"""Seeded synthetic meshes: the unit-cube PEC cavity cut into n^3 hexahedra,
each hexahedron split into the six Kuhn tetrahedra that share its main
diagonal.

This module only produces input arrays (vertex coordinates and tetrahedron
vertex lists).  It holds none of the finite-element arithmetic: no basis
functions, no element matrices, no assembly.

Numbering (fixed, so that per-tetrahedron seeded arrays are reproducible):
  * vertex (i, j, k), 0 <= i, j, k <= n, has id (i*(n+1) + j)*(n+1) + k and
    coordinates (i/n, j/n, k/n), optionally graded per axis as x -> x**grade;
  * hexahedron (i, j, k), 0 <= i, j, k < n, has id (i*n + j)*n + k;
  * hexahedron h is split into 6 tetrahedra, one per permutation p of the
    axes in lexicographic order (012, 021, 102, 120, 201, 210): the
    tetrahedron walks v0 = (i, j, k), v_{m+1} = v_m + unit(p_m); its id is
    6*h + index(p).
Every hexahedron is cut along the same diagonal, so the mesh is conforming.
"""
from __future__ import annotations

import itertools

import numpy as np

PERMS = tuple(itertools.permutations(range(3)))  # lexicographic order


def vertex_id(i, j, k, n):
    return (i * (n + 1) + j) * (n + 1) + k


def cube_mesh(n: int, grade: float = 1.0):
    """Return (coords [n_v, 3] float64, tets [n_t, 4] int32, hex_of_tet [n_t])."""
    if n < 1:
        raise ValueError("n must be >= 1")
    t = np.arange(n + 1, dtype=np.float64) / n
    if grade != 1.0:
        t = t ** grade
    I, J, K = np.meshgrid(t, t, t, indexing="ij")
    coords = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)

    hi, hj, hk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    hi, hj, hk = hi.ravel(), hj.ravel(), hk.ravel()
    n_hex = n ** 3
    tets = np.empty((n_hex, 6, 4), dtype=np.int64)
    for pi, p in enumerate(PERMS):
        v = [hi.copy(), hj.copy(), hk.copy()]
        tets[:, pi, 0] = vertex_id(v[0], v[1], v[2], n)
        for m in range(3):
            v[p[m]] = v[p[m]] + 1
            tets[:, pi, m + 1] = vertex_id(v[0], v[1], v[2], n)
    tets = tets.reshape(n_hex * 6, 4).astype(np.int32)
    hex_of_tet = np.repeat(np.arange(n_hex, dtype=np.int64), 6)
    return coords, tets, hex_of_tet


def hex_ijk(n: int):
    """(i, j, k) index of every hexahedron in id order, each as an int array."""
    hi, hj, hk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return hi.ravel(), hj.ravel(), hk.ravel()


def mesh_edges(tets: np.ndarray):
    """Unique vertex pairs (lo, hi), lexicographically sorted.

    Topology only (used to size and place seeded source arrays); the solver
    and the oracle each derive their own edge lists.
    """
    s = np.sort(tets.astype(np.int64), axis=1)
    pairs = np.concatenate([s[:, [a, b]] for a, b in
                            ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))])
    key = np.unique(pairs[:, 0] * (int(s.max()) + 1) + pairs[:, 1])
    nv = int(s.max()) + 1
    return np.stack([key // nv, key % nv], axis=1)


def boundary_edge_mask(coords: np.ndarray, edges: np.ndarray):
    """True for edges whose two end points lie on one face of the unit cube."""
    a, b = coords[edges[:, 0]], coords[edges[:, 1]]
    on = np.zeros(len(edges), dtype=bool)
    for ax in range(3):
        for val in (0.0, 1.0):
            on |= (a[:, ax] == val) & (b[:, ax] == val)
    return on


def jittered_cube_mesh(n: int, amp: float, seed: int):
    """cube_mesh(n) with every vertex strictly inside the cube moved by a
    seeded uniform offset in [-amp/n, amp/n]^3 (boundary vertices stay, so
    the outer surface is still the unit cube).  amp <= 0.2 keeps every
    tetrahedron positively oriented."""
    coords, tets, hx = cube_mesh(n)
    rng = np.random.default_rng(seed)
    inner = np.all((coords > 0.0) & (coords < 1.0), axis=1)
    coords = coords.copy()
    coords[inner] += rng.uniform(-amp / n, amp / n, size=(int(inner.sum()), 3))
    return coords, tets, hx


def centred_cube_mesh(n: int):
    """The n^3 hexahedra each cut into 12 tetrahedra around an added centre
    vertex: every face is split into two triangles along the diagonal through
    its vertex of smallest id (the same choice from both sides, so the mesh
    is conforming), and each triangle is joined to the centre.  Edges meet
    more tetrahedra than in the Kuhn split, so rows of the edge matrices are
    longer: up to 25 nonzeros, against 19 for the Kuhn split.

    Returns (coords, tets, hex_of_tet); centre of hexahedron h has vertex id
    (n+1)^3 + h; tetrahedra of hexahedron h are 12h .. 12h+11.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    coords, _, _ = cube_mesh(n)
    hi, hj, hk = hex_ijk(n)
    centres = np.stack([hi + 0.5, hj + 0.5, hk + 0.5], axis=1) / n
    coords = np.concatenate([coords, centres])
    nv0 = (n + 1) ** 3
    # faces of a unit cube as corner offsets in cyclic order
    faces = (
        ((0, 0, 0), (0, 1, 0), (0, 1, 1), (0, 0, 1)),
        ((1, 0, 0), (1, 1, 0), (1, 1, 1), (1, 0, 1)),
        ((0, 0, 0), (1, 0, 0), (1, 0, 1), (0, 0, 1)),
        ((0, 1, 0), (1, 1, 0), (1, 1, 1), (0, 1, 1)),
        ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0)),
        ((0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)),
    )
    n_hex = n ** 3
    tets = np.empty((n_hex, 12, 4), dtype=np.int64)
    c = nv0 + np.arange(n_hex)
    t = 0
    for f in faces:
        q = np.stack([vertex_id(hi + a, hj + b, hk + d, n) for a, b, d in f], axis=1)  # [n_hex, 4]
        m = np.argmin(q, axis=1)                      # diagonal through the smallest id
        rows = np.arange(n_hex)
        v0 = q[rows, m]
        v1 = q[rows, (m + 1) % 4]
        v2 = q[rows, (m + 2) % 4]
        v3 = q[rows, (m + 3) % 4]
        tets[:, t] = np.stack([c, v0, v1, v2], axis=1)
        tets[:, t + 1] = np.stack([c, v0, v2, v3], axis=1)
        t += 2
    tets = tets.reshape(n_hex * 12, 4).astype(np.int32)
    return coords, tets, np.repeat(np.arange(n_hex, dtype=np.int64), 12)
