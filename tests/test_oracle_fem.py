"""Pins of the oracle's spatial discretisation (edges, Whitney element
matrices, assembly) against facts that do not come from its own formulas:
closed-form counts, exact element values worked out by hand from the
definition of the Whitney 1-form basis (Sec. II-B-1), an independent
quadrature of the basis, the discrete de Rham property curl grad = 0, and
the closed-form eigenfrequencies of the PEC unit-cube cavity."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle.fem import Discretisation, LOCAL_EDGES, canonical_edges, element_matrices, pec_mask
from workloads.mesh import cube_mesh


# --------------------------------------------------------------------------
# counts
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_edge_counts_closed_form(n):
    """n^3 Kuhn-cut cube: axis edges 3n(n+1)^2, one diagonal per square face
    3n^2(n+1), one per hexahedron n^3.  The boundary is a triangulated sphere
    with V = 6n^2+2 vertices and F = 12n^2 triangles, so Euler's formula
    gives 18n^2 boundary edges."""
    c, t, _ = cube_mesh(n)
    edges, te = canonical_edges(t)
    n_e = 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3
    assert len(edges) == n_e
    assert (edges[:, 0] < edges[:, 1]).all()
    key = edges[:, 0] * (len(c) + 1) + edges[:, 1]
    assert (np.diff(key) > 0).all()                       # lexicographic
    assert pec_mask(c, edges).sum() == 18 * n * n
    assert te.shape == (6 * n ** 3, 6)


def test_survey_sizes_match():
    """Sizes of the 8^3 cavity quoted for the small FP64 workload."""
    c, t, _ = cube_mesh(8)
    d = Discretisation(c, t)
    assert (d.n_e, d.n_int) == (4184, 3032)


# --------------------------------------------------------------------------
# element matrices: exact values worked out by hand
# --------------------------------------------------------------------------
# Reference tetrahedron (0,0,0),(1,0,0),(0,1,0),(0,0,1), eps = mu = 1, edge
# order 01,02,03,12,13,23.  grad lam = (-1,-1,-1),(1,0,0),(0,1,0),(0,0,1),
# V = 1/6.  Hand checks: T[01,01] = (V/20)(2*1 + 1 + 1 + 2*3) = 1/12 and
# S[01,01] = 4 V |g0 x g1|^2 = 4 (1/6) 2 = 4/3.
REF_T360 = [[30, 15, 15, 0, 0, 0], [15, 30, 15, 0, 0, 0], [15, 15, 30, 0, 0, 0],
            [0, 0, 0, 12, 3, -3], [0, 0, 0, 3, 12, 3], [0, 0, 0, -3, 3, 12]]
REF_S3 = [[4, -2, -2, 2, 2, 0], [-2, 4, -2, -2, 0, 2], [-2, -2, 4, 0, -2, -2],
          [2, -2, 0, 2, 0, 0], [2, 0, -2, 0, 2, 0], [0, 2, -2, 0, 0, 2]]
# Kuhn tetrahedron (0,0,0),(1,0,0),(1,1,0),(1,1,1): lam = 1-x, x-y, y-z, z,
# grad lam = (-1,0,0),(1,-1,0),(0,1,-1),(0,0,1), V = 1/6.  Hand checks:
# T[01,01] = (V/20)(2*2 + 1 + 1 + 2*1) = 1/15, T[01,02] = (V/20)(2(-1)+1-0+1) = 0,
# T[01,12] = (V/20)(-1 - 2 - 0 - 1) = -1/30, S[12,12] = 4V|(1,1,1)|^2 = 2,
# S[01,12] = 4V (0,0,1).(1,1,1) = 2/3.
KUHN_T360 = [[24, 0, 6, -12, -9, 3], [0, 18, -3, 3, -3, -9], [6, -3, 12, -6, -3, 6],
             [-12, 3, -6, 30, 3, -12], [-9, -3, -3, 3, 18, 0], [3, -9, 6, -12, 0, 24]]
KUHN_S3 = [[2, -2, 0, 2, 0, 0], [-2, 4, -2, -4, 2, 0], [0, -2, 2, 2, -2, 0],
           [2, -4, 2, 6, -4, 2], [0, 2, -2, -4, 4, -2], [0, 0, 0, 2, -2, 2]]

REF = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
KUHN = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1]], dtype=float)


@pytest.mark.parametrize("X,T360,S3", [(REF, REF_T360, REF_S3), (KUHN, KUHN_T360, KUHN_S3)])
def test_element_matrices_exact(X, T360, S3):
    Te, Se = element_matrices(X, np.array([[0, 1, 2, 3]]))
    np.testing.assert_allclose(Te[0] * 360.0, np.array(T360, float), atol=1e-13)
    np.testing.assert_allclose(Se[0] * 3.0, np.array(S3, float), atol=1e-13)


def _whitney_by_quadrature(X, eps=1.0, mu=1.0):
    """Independent route: evaluate W_ij = lam_i grad lam_j - lam_j grad lam_i
    at the points of a degree-2-exact 4-point rule (W.W is quadratic), with
    lam from solving the affine map and grad lam / curl W from central
    differences (exact for affine/linear fields up to rounding)."""
    D = (X[1:] - X[0]).T

    def lam(x):
        l123 = np.linalg.solve(D, x - X[0])
        return np.concatenate([[1.0 - l123.sum()], l123])

    h = 1e-3
    grad = np.array([[(lam(X[0] + h * ei)[k] - lam(X[0] - h * ei)[k]) / (2 * h)
                      for ei in np.eye(3)] for k in range(4)])

    def W(x, e):
        i, j = LOCAL_EDGES[e]
        l = lam(x)
        return l[i] * grad[j] - l[j] * grad[i]

    def curlW(x, e):
        J = np.array([(W(x + h * ei, e) - W(x - h * ei, e)) / (2 * h) for ei in np.eye(3)]).T
        return np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])

    V = abs(np.linalg.det(D)) / 6.0
    a, b = 0.5854101966249685, 0.1381966011250105
    pts = [X.T @ np.roll([a, b, b, b], k) for k in range(4)]
    T = np.zeros((6, 6)); S = np.zeros((6, 6))
    for p in pts:
        for A in range(6):
            for B in range(6):
                T[A, B] += eps * V / 4 * W(p, A) @ W(p, B)
                S[A, B] += V / 4 / mu * curlW(p, A) @ curlW(p, B)
    return T, S


def test_element_matrices_vs_quadrature_random_tets():
    rng = np.random.default_rng(11)
    for _ in range(5):
        X = rng.uniform(-1, 1, (4, 3))
        eps, mu = rng.uniform(1, 4), rng.uniform(0.5, 2)
        Te, Se = element_matrices(X, np.array([[0, 1, 2, 3]]), [eps], [mu])
        Tq, Sq = _whitney_by_quadrature(X, eps, mu)
        scale = np.abs(Tq).max()
        np.testing.assert_allclose(Te[0], Tq, atol=1e-9 * scale)
        np.testing.assert_allclose(Se[0], Sq, atol=1e-8 * np.abs(Sq).max())


def test_exact_rationals_hand_formula():
    """Exact rational evaluation of the reference-tet mass entries from
    integral lam_a lam_b = V (1 + delta_ab)/20 (Fraction arithmetic)."""
    g = [(-1, -1, -1), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    V = Fraction(1, 6)
    dot = lambda u, v: sum(Fraction(a) * b for a, b in zip(u, v))
    m = lambda a, b: V * (2 if a == b else 1) / 20
    for A, (i, j) in enumerate(LOCAL_EDGES):
        for B, (k, l) in enumerate(LOCAL_EDGES):
            val = (m(i, k) * dot(g[j], g[l]) - m(i, l) * dot(g[j], g[k])
                   - m(j, k) * dot(g[i], g[l]) + m(j, l) * dot(g[i], g[k]))
            assert val * 360 == REF_T360[A][B]


# --------------------------------------------------------------------------
# de Rham: curl grad = 0, kernel dimension
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,grade", [(4, 1.0), (5, 1.5)])
def test_curl_grad_zero(n, grade):
    c, t, _ = cube_mesh(n, grade)
    rng = np.random.default_rng(3)
    d = Discretisation(c, t, eps=rng.uniform(1, 4, len(t)), mu=rng.uniform(0.5, 2, len(t)))
    G = d.gradient()
    SG = d.S @ G
    assert abs(SG).max() <= 1e-13 * abs(d.S).max()
    # the gradient of a nodal function is a Whitney field: T G != 0
    assert abs(d.T @ G).max() > 1e-3 * abs(d.T).max()


def test_de_rham_on_centred_mesh():
    """The same two facts on another topology (cubes cut into 12 tetrahedra
    around an added centre): S G = 0, and dim ker S = number of interior
    vertices = (n-1)^3 grid vertices + n^3 centres."""
    from workloads.mesh import centred_cube_mesh
    n = 3
    c, t, _ = centred_cube_mesh(n)
    rng = np.random.default_rng(5)
    d = Discretisation(c, t, eps=rng.uniform(1, 4, len(t)), mu=rng.uniform(0.5, 2, len(t)))
    G = d.gradient()
    assert abs(d.S @ G).max() <= 1e-13 * abs(d.S).max()
    w = np.linalg.eigvalsh(Discretisation(c, t).S.toarray())
    assert (np.abs(w) < 1e-10 * w.max()).sum() == (n - 1) ** 3 + n ** 3


def test_kernel_dimension():
    """dim ker S = number of interior vertices = (n-1)^3."""
    n = 3
    c, t, _ = cube_mesh(n)
    d = Discretisation(c, t)
    w = np.linalg.eigvalsh(d.S.toarray())
    zero = (np.abs(w) < 1e-10 * w.max()).sum()
    assert zero == (n - 1) ** 3


# --------------------------------------------------------------------------
# PEC cavity eigenfrequencies: k^2 = pi^2 (l^2 + m^2 + p^2), O(h^2)
# --------------------------------------------------------------------------
def _cavity_modes(n, count):
    c, t, _ = cube_mesh(n)
    d = Discretisation(c, t)
    w = sla.eigh(d.S.toarray(), d.T.toarray(), eigvals_only=True)
    return np.sort(w[w > 1e-6])[:count] / np.pi ** 2


def test_cavity_eigenvalues_converge():
    """The exact cube-cavity spectrum is pi^2 {2 (x3), 3 (x2), 5 (x6), ...};
    on the Kuhn mesh the degenerate groups split, but every value converges
    at second order in h: errors at n = 4 and n = 6 differ by (6/4)^2."""
    exact = np.array([2, 2, 2, 3, 3, 5, 5, 5, 5, 5, 5])
    e4 = _cavity_modes(4, 11)
    e6 = _cavity_modes(6, 11)
    err4 = np.abs(e4 - exact)
    err6 = np.abs(e6 - exact)
    assert err6.max() < 0.25
    ratio = err4.max() / err6.max()
    assert 1.8 < ratio < 2.8, ratio
    # multiplicities of the split triple and pair survive: 2.02.. twice, 3.06.. twice
    assert abs(e4[1] - e4[2]) < 1e-10 and abs(e4[3] - e4[4]) < 1e-10
