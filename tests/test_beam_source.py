"""The beam source is charge conserving (Sec. II-A): for every interior
vertex k, dt (G^T J^{n+1/2})_k equals sum_p q_p (lam_k(b_p) - lam_k(a_p)),
the change of the nodal charge of the delta-shaped particles, with lam_k the
nodal hat function evaluated independently (containing tetrahedron found by
brute force, barycentric coordinates by a linear solve)."""
import numpy as np

from oracle.fem import Discretisation
from workloads.beam import BeamSampler, beam_source, deposit
from workloads.mesh import cube_mesh, mesh_edges


def _hat(coords, tets, x):
    """lam_k(x) for every vertex k (dense vector)."""
    out = np.zeros(len(coords))
    for t in tets:
        X = coords[t]
        D = (X[1:] - X[0]).T
        l = np.linalg.solve(D, x - X[0])
        lam = np.concatenate([[1 - l.sum()], l])
        if lam.min() >= -1e-12:
            out[t] = lam
            return out
    raise AssertionError("point outside mesh")


def test_deposit_conserves_charge():
    n = 3
    c, t, _ = cube_mesh(n)
    edges = mesh_edges(t)
    keys = edges[:, 0] * len(c) + edges[:, 1]
    rng = np.random.default_rng(0)
    m = 40
    a = rng.uniform(0.05, 0.95, (m, 3))
    b = a + rng.uniform(-0.25, 0.25, (m, 3)) / n       # shorter than a cell
    b = np.clip(b, 0.01, 0.99)
    q = rng.choice([-1.0, 1.0], m) * rng.uniform(0.5, 2, m)
    dt = 0.1
    J = deposit(n, keys, len(c), a, b, q, dt, len(edges))
    d = Discretisation(c, t)
    G = d.gradient()
    lhs = dt * (G.T @ J[d.interior])
    nodes = d.interior_nodes()
    rhs = np.zeros(len(nodes))
    for p in range(m):
        rhs += q[p] * (_hat(c, t, b[p]) - _hat(c, t, a[p]))[nodes]
    np.testing.assert_allclose(lhs, rhs, atol=1e-12 * np.abs(q).sum())
    assert np.abs(rhs).max() > 1e-3


def test_closed_loop_deposits_no_charge():
    n = 2
    c, t, _ = cube_mesh(n)
    edges = mesh_edges(t)
    keys = edges[:, 0] * len(c) + edges[:, 1]
    pts = np.array([[0.3, 0.3, 0.3], [0.6, 0.35, 0.4], [0.55, 0.7, 0.45], [0.3, 0.3, 0.3]])
    J = deposit(n, keys, len(c), pts[:-1], pts[1:], np.ones(3), 1.0, len(edges))
    d = Discretisation(c, t)
    assert np.abs(d.gradient().T @ J[d.interior]).max() < 1e-13
    assert np.abs(J).max() > 1e-3


def test_beam_source_wraps_and_conserves():
    """Small beam crossing the z = 1 wall: interior Gauss increments still
    match the nodal charge change, wall vertices excluded."""
    n = 4
    c, t, _ = cube_mesh(n)
    edges = mesh_edges(t)
    dt = 0.1
    bs = BeamSampler(n, 30, 0.2, 0.01, 0.3, 1.0, seed=5)
    J = beam_source(c, t, edges, n, 2, dt, 1, particles=30, radius=0.2, vth=0.01, vz=0.3,
                    q0=1.0, seed=5, steps=[3])
    d = Discretisation(c, t)
    lhs = dt * (d.gradient().T @ J[0, 0][d.interior])
    nodes = d.interior_nodes()
    pa, pb = bs.positions(3 * dt), bs.positions(4 * dt)
    rhs = np.zeros(len(nodes))
    for p in range(30):
        rhs += bs.q[p] * (_hat(c, t, pb[p]) - _hat(c, t, pa[p]))[nodes]
    np.testing.assert_allclose(lhs, rhs, atol=1e-12 * 30)
