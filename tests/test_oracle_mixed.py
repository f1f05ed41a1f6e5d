"""Pins of the mixed E/B oracle (oracle/mixed.py) against facts that do not
come from its own formulas: the 2-form mass and the curl incidence
reproduce the independently built curl-curl matrix (S = C^T M C); the
divergence of a curl vanishes exactly (D C = 0 with D from the geometric
outward normals); Euler's formula for the face count; the flux of a 2-form
basis function through its own face is one and through the other faces of
its tetrahedron zero; the trapezoid step conserves the discrete energy; and
eliminating b reproduces the edge-only Newmark recurrence with beta = 1/4
(the oracle of that form)."""
import numpy as np
import pytest

from oracle.fem import barycentric_gradients, sort_tets
from oracle.mixed import LOCAL_FACES, MixedOracle, canonical_faces, curl_incidence
from oracle.newmark import NewmarkOracle
from workloads.mesh import cube_mesh, jittered_cube_mesh
from workloads.sources import dense_random_source


@pytest.fixture(scope="module")
def jm():
    c, t, _ = jittered_cube_mesh(3, 0.2, 4)
    mu = np.random.default_rng(3).uniform(1, 2, len(t))
    return c, t, mu


def test_curl_curl_from_face_mass(jm):
    c, t, mu = jm
    o = MixedOracle(c, t, mu=mu, dt=0.1)
    S2 = (o.C.T @ o.M @ o.C).toarray()
    S = o.d.S.toarray()
    assert np.abs(S2 - S).max() <= 1e-12 * np.abs(S).max()


def test_curl_curl_from_face_mass_centred_mesh():
    """S = C^T M C also on the centred-cube topology (faces of 12-tetrahedron
    cubes, diagonals chosen by the smallest vertex id)."""
    from workloads.mesh import centred_cube_mesh
    c, t, _ = centred_cube_mesh(2)
    mu = np.random.default_rng(9).uniform(1, 2, len(t))
    o = MixedOracle(c, t, mu=mu, dt=0.1, factor=False)
    S2 = (o.C.T @ o.M @ o.C).toarray()
    S = o.d.S.toarray()
    assert np.abs(S2 - S).max() <= 1e-12 * np.abs(S).max()


def test_divergence_of_curl_is_zero(jm):
    c, t, mu = jm
    faces, tf = canonical_faces(t)
    st = sort_tets(t)
    from oracle.fem import canonical_edges
    edges, _ = canonical_edges(t)
    C = curl_incidence(edges, faces)
    D = np.zeros((len(t), len(faces)))
    for k in range(len(t)):
        xc = c[st[k]].mean(axis=0)
        for f in tf[k]:
            a, b, d = c[faces[f]]
            nrm = np.cross(b - a, d - a)
            D[k, f] = 1.0 if nrm @ ((a + b + d) / 3 - xc) > 0 else -1.0
    e = np.random.default_rng(1).normal(size=len(edges))
    assert np.abs(D @ (C @ e)).max() <= 1e-12
    assert np.abs(C @ e).max() > 0.1


@pytest.mark.parametrize("n", [1, 2, 4])
def test_face_count_euler(n):
    c, t, _ = cube_mesh(n)
    faces, _ = canonical_faces(t)
    from oracle.fem import canonical_edges
    edges, _ = canonical_edges(t)
    assert len(c) - len(edges) + len(faces) - len(t) == 1


def test_face_flux_is_kronecker(jm):
    c, t, mu = jm
    g, vol = barycentric_gradients(c, t)
    st = sort_tets(t)
    for k in range(0, len(t), 7):
        x = c[st[k]]
        for F, fv in enumerate(LOCAL_FACES):
            i, j, l = fv
            cf = {i: np.cross(g[k, j], g[k, l]), j: np.cross(g[k, l], g[k, i]), l: np.cross(g[k, i], g[k, j])}
            for G, gv in enumerate(LOCAL_FACES):
                lam = np.zeros(4)
                lam[list(gv)] = 1.0 / 3.0                       # centroid of face G
                W = 2.0 * sum(lam[a] * v for a, v in cf.items())
                p, q, r = x[list(gv)]
                flux = W @ (0.5 * np.cross(q - p, r - p))       # area-weighted normal i -> j -> k
                assert abs(flux - (1.0 if F == G else 0.0)) <= 1e-12


def test_trapezoid_conserves_energy(jm):
    c, t, mu = jm
    o = MixedOracle(c, t, mu=mu, dt=0.2)
    rng = np.random.default_rng(2)
    e0 = rng.normal(size=(2, o.d.n_e)); e0[:, o.d.pec] = 0.0
    b0 = rng.normal(size=(2, o.n_f))
    E, B = o.run(np.zeros((12, 2, o.d.n_e)), e0, b0)
    H = np.array([o.energy(E[k], B[k]) for k in range(len(E))])
    assert np.abs(H - H[0]).max() <= 1e-12 * H[0].max()
    assert np.abs(E[-1] - E[0]).max() > 1e-2


def test_eliminating_b_gives_newmark_quarter():
    c, t, _ = cube_mesh(4)
    dt, N = 0.05, 8
    eps = np.random.default_rng(4).uniform(1, 3, len(t))
    m = MixedOracle(c, t, eps=eps, dt=dt)
    J = dense_random_source(m.d.n_e, ~m.d.pec, N, dt, 0.15, 0.05, seed=5, nrhs=2)
    Em, _ = m.run(J)
    En = NewmarkOracle(c, t, eps=eps, dt=dt, beta=0.25).run(J)
    assert np.abs(Em - En).max() <= 1e-11 * np.abs(En).max()
    assert np.abs(En).max() > 1e-3


def test_property_checks_vanish_on_oracle_steps(jm):
    """The any-size properties used at full size: zero (to rounding) on the
    oracle's own steps, large for a perturbed field."""
    c, t, mu = jm
    o = MixedOracle(c, t, mu=mu, dt=0.1)
    rng = np.random.default_rng(8)
    J = dense_random_source(o.d.n_e, ~o.d.pec, 3, 0.1, 0.15, 0.05, seed=6, nrhs=2)
    E, B = o.run(J)
    for k in range(3):
        assert o.eliminated_residual(E[k + 1], E[k], B[k], J[k]).max() <= 1e-12
        assert o.face_update_residual(E[k + 1], E[k], B[k], B[k + 1]).max() <= 1e-13 * np.abs(B[k + 1]).max()
    bad = E[2] + 1e-6 * rng.normal(size=E[2].shape) * (~o.d.pec)
    assert o.eliminated_residual(bad, E[1], B[1], J[1]).max() > 1e-8
    assert o.face_update_residual(bad, E[1], B[1], B[2]).max() > 1e-9
