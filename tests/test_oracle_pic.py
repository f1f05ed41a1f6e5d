"""Pins of the particle-step oracle (oracle/pic.py) against facts that do not
come from its own formulas: Whitney forms reproduce constant fields and their
curls reproduce the curl of a linear potential exactly (Sec. II-B-1); the
line integral of an edge function along its own edge is one and along the
others zero; the exact current mapping of Sec. II-A satisfies the discrete
continuity equation with the hat functions evaluated by an independent
linear solve; the deposit is additive over a split path and odd under path
reversal; it agrees with the structured (plane-splitting) beam deposit on
the Kuhn mesh; Adams-Bashforth reproduces the closed-form motion under a
constant force and converges at second order on a gyration orbit."""
import numpy as np
import pytest

from oracle import pic
from workloads.beam import deposit as kuhn_deposit
from workloads.mesh import centred_cube_mesh, cube_mesh, jittered_cube_mesh


@pytest.fixture(scope="module")
def jmesh():
    c, t, _ = jittered_cube_mesh(3, 0.2, 7)
    return pic.TetMesh(c, t)


def _inside_points(rng, m, margin=0.05):
    return rng.uniform(margin, 1.0 - margin, size=(m, 3))


def _hat_values(mesh, x):
    """lam of the containing tet's 4 vertices at x, from solving
    [x_v; 1] w = [x; 1] (not from the stored gradients)."""
    t = pic.locate(mesh, x[None, :])[0]
    assert t >= 0
    V = mesh.coords[mesh.st[t]]                       # [4, 3]
    A = np.vstack([V.T, np.ones(4)])
    w = np.linalg.solve(A, np.append(x, 1.0))
    return mesh.st[t], w


def test_locate_brute_force(jmesh):
    rng = np.random.default_rng(0)
    X = _inside_points(rng, 40, 0.0)
    T = pic.locate(jmesh, X)
    assert (T >= 0).all()
    for x, t in zip(X, T):
        _, w = _hat_values(jmesh, x)
        assert w.min() >= -1e-12
    assert pic.locate(jmesh, np.array([[1.2, 0.5, 0.5]]))[0] == -1


def test_whitney_reproduces_constant_field(jmesh):
    rng = np.random.default_rng(1)
    E0 = np.array([0.3, -1.2, 0.7])
    x = jmesh.coords
    e = (x[jmesh.edges[:, 1]] - x[jmesh.edges[:, 0]]) @ E0   # line integrals
    X = _inside_points(rng, 50)
    E = pic.whitney_field(jmesh, e, pic.locate(jmesh, X), X)
    np.testing.assert_allclose(E, np.broadcast_to(E0, E.shape), rtol=0, atol=1e-13)


def test_curl_of_linear_potential(jmesh):
    """A = (B0 x r)/2 + c has curl B0; its edge integrals are exact at the
    edge midpoint because A is linear."""
    B0 = np.array([0.4, 0.9, -0.5])
    c0 = np.array([0.1, 0.2, -0.3])
    x = jmesh.coords
    a, b = x[jmesh.edges[:, 0]], x[jmesh.edges[:, 1]]
    mid = 0.5 * (a + b)
    A = 0.5 * np.cross(B0, mid) + c0
    e = np.einsum("ed,ed->e", A, b - a)
    curl = pic.tet_curl(jmesh, e)
    np.testing.assert_allclose(curl, np.broadcast_to(B0, curl.shape), rtol=0, atol=1e-12)
    B1 = pic.faraday(jmesh, e, np.ones_like(curl), -0.5)
    np.testing.assert_allclose(B1, 1.0 - 0.5 * B0[None, :] + 0 * B1, atol=1e-12)


def test_deposit_along_an_edge_is_unit(jmesh):
    """int W_e . dl over edge e is 1 and over every other edge 0, so a
    charge q moving along edge e in dt deposits J = q/dt on e only."""
    rng = np.random.default_rng(2)
    c = jmesh.coords
    inner = np.all((c > 0) & (c < 1), axis=1)
    cand = np.flatnonzero(inner[jmesh.edges[:, 0]] & inner[jmesh.edges[:, 1]])
    for e in rng.choice(cand, 4, replace=False):
        i, j = jmesh.edges[e]
        J = pic.deposit(jmesh, c[i], c[j], 2.0, 0.5)
        ref = np.zeros(jmesh.n_e)
        ref[e] = 4.0
        np.testing.assert_allclose(J, ref, rtol=0, atol=1e-12)


@pytest.fixture(scope="module")
def cmesh():
    c, t, _ = centred_cube_mesh(3)
    return pic.TetMesh(c, t)


@pytest.mark.parametrize("which", ["jittered", "centred"])
def test_deposit_discrete_continuity(jmesh, cmesh, which):
    """dt * sum_{e at k} sign(e, k) J_e = q (lam_k(b) - lam_k(a)) at every
    vertex k (sign +1 at the higher end): the charge that leaves the
    hat function of k is the current through the edges at k.  Also on the
    centred-cube topology (vertices in up to 24 tetrahedra)."""
    jmesh = jmesh if which == "jittered" else cmesh
    rng = np.random.default_rng(3)
    m = 30
    A = _inside_points(rng, m)
    B = A + rng.normal(0, 0.15, size=(m, 3))
    B = np.clip(B, 0.01, 0.99)
    q = rng.choice([-1.0, 1.0], m) * rng.uniform(0.5, 2.0, m)
    dt = 0.3
    J = pic.deposit(jmesh, A, B, q, dt)
    nv = len(jmesh.coords)
    div = np.zeros(nv)
    np.add.at(div, jmesh.edges[:, 1], J * dt)
    np.add.at(div, jmesh.edges[:, 0], -J * dt)
    ref = np.zeros(nv)
    for p in range(m):
        vb, wb = _hat_values(jmesh, B[p])
        va, wa = _hat_values(jmesh, A[p])
        np.add.at(ref, vb, q[p] * wb)
        np.add.at(ref, va, -q[p] * wa)
    np.testing.assert_allclose(div, ref, rtol=0, atol=1e-12)
    assert np.abs(ref).max() > 0.1


def test_deposit_additive_and_odd(jmesh):
    rng = np.random.default_rng(4)
    a, b = _inside_points(rng, 2)
    s = 0.37
    m = a + s * (b - a)
    J = pic.deposit(jmesh, a, b, 1.0, 1.0)
    J2 = pic.deposit(jmesh, a, m, 1.0, 1.0) + pic.deposit(jmesh, m, b, 1.0, 1.0)
    np.testing.assert_allclose(J2, J, rtol=0, atol=1e-13)
    np.testing.assert_allclose(pic.deposit(jmesh, b, a, 1.0, 1.0), -J, rtol=0, atol=1e-13)
    # a path inside one tetrahedron that stays put deposits nothing
    np.testing.assert_allclose(pic.deposit(jmesh, a, a, 1.0, 1.0), 0.0, atol=0)


def test_deposit_matches_structured_kuhn_deposit():
    """Brute-force piece search vs the hexahedron/Kuhn-plane splitting of the
    beam source generator (a different algorithm) on a regular mesh.  That
    generator cuts each axis at most once, so paths move less than one cell
    per axis."""
    n = 4
    c, t, _ = cube_mesh(n)
    mesh = pic.TetMesh(c, t)
    rng = np.random.default_rng(5)
    m = 60
    A = _inside_points(rng, m, 0.02)
    B = np.clip(A + rng.uniform(-0.9 / n, 0.9 / n, size=(m, 3)), 0.01, 0.99)
    q = rng.uniform(-1, 1, m)
    dt = 0.01
    J = pic.deposit(mesh, A, B, q, dt)
    nv1 = len(c)
    keys = mesh.edges[:, 0] * nv1 + mesh.edges[:, 1]
    K = kuhn_deposit(n, keys, nv1, A, B, q, dt, mesh.n_e)
    np.testing.assert_allclose(J, K, rtol=0, atol=1e-11 * np.abs(K).max())


def test_push_constant_force_closed_form():
    """Constant acceleration a: Euler start then AB2 gives v_n = v0 + n dt a
    exactly and x_n = x0 + n dt v0 + (n^2 - 1) dt^2 a / 2."""
    x0 = np.array([[0.1, 0.2, 0.3], [0.5, 0.5, 0.5]])
    v0 = np.array([[1.0, 0.0, -1.0], [0.2, 0.3, 0.4]])
    E = np.array([[0.5, -0.25, 2.0], [1.0, 1.0, 1.0]])
    qm = np.array([2.0, -1.0])
    acc = qm[:, None] * E
    dt, n = 0.01, 25
    x, v, hv, ha = x0.copy(), v0.copy(), None, None
    for k in range(n):
        a = pic.lorentz(qm, E, np.zeros_like(E), v)
        x, v, hv, ha = pic.push_ab2(x, v, a, hv, ha, dt, k == 0)
    np.testing.assert_allclose(v, v0 + n * dt * acc, rtol=0, atol=1e-14)
    np.testing.assert_allclose(x, x0 + n * dt * v0 + 0.5 * (n * n - 1) * dt * dt * acc, rtol=0, atol=1e-14)


def test_push_gyration_second_order():
    """Uniform B, no E: the exact orbit is a circle at the cyclotron
    frequency qB/m; the AB2 error at a fixed time falls ~4x per halving."""
    Bz, qm = 2.0, 1.5
    v0 = np.array([[0.3, 0.0, 0.1]])
    x0 = np.array([[0.0, 0.0, 0.0]])
    T = 1.0
    w = qm * Bz

    def exact(t):
        # v' = qm v x B with B = Bz z: vx' = w vy, vy' = -w vx
        vx = 0.3 * np.cos(w * t)
        vy = -0.3 * np.sin(w * t)
        x = 0.3 * np.sin(w * t) / w
        y = 0.3 * (np.cos(w * t) - 1.0) / w
        return np.array([x, y, 0.1 * t]), np.array([vx, vy, 0.1])

    errs = []
    for n in (100, 200, 400):
        dt = T / n
        x, v, hv, ha = x0.copy(), v0.copy(), None, None
        B = np.array([[0.0, 0.0, Bz]])
        for k in range(n):
            a = pic.lorentz(np.array([qm]), np.zeros((1, 3)), B, v)
            x, v, hv, ha = pic.push_ab2(x, v, a, hv, ha, dt, k == 0)
        xe, ve = exact(T)
        errs.append(np.abs(x[0] - xe).max() + np.abs(v[0] - ve).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs
