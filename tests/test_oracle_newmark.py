"""Pins of the oracle's time stepping (Sec. II-B-2) and its adjoint against
closed forms and invariants of the scheme:
  * one cavity mode evolves as cos(n theta) with cos(theta) =
    (1 - (1/2 - beta) k^2 dt^2) / (1 + beta k^2 dt^2)  (Newmark, gamma = 1/2);
  * without sources the discrete energy H^{n+1/2} is constant (beta = 1/4,
    the unconditionally stable choice);
  * the discrete Gauss law G^T T e^n + q^n = 0 holds to rounding for the
    time-integrated current of Sec. II-A (charge conservation, Sec. IV-B);
  * the direct solve agrees with a dense LAPACK solve;
  * the adjoint passes the dot-product test and central differences."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.newmark import NewmarkOracle
from workloads.mesh import cube_mesh
from workloads.sources import dense_random_source


def _oracle(n=3, dt=0.05, beta=0.25, seed=None, grade=1.0):
    c, t, _ = cube_mesh(n, grade)
    eps = None if seed is None else np.random.default_rng(seed).uniform(1, 4, len(t))
    return NewmarkOracle(c, t, eps=eps, dt=dt, beta=beta)


@pytest.mark.parametrize("beta,dt", [(0.25, 0.05), (0.25, 0.4), (0.3, 0.1)])
def test_single_mode_closed_form(beta, dt):
    o = _oracle(4, dt=dt, beta=beta)
    w, V = sla.eigh(o.d.S.toarray(), o.d.T.toarray())
    v = V[:, -1]                                  # stiffest mode
    k2 = w[-1]
    c = (1 - (0.5 - beta) * k2 * dt * dt) / (1 + beta * k2 * dt * dt)
    theta = np.arccos(c)
    if beta == 0.25:
        assert abs(theta - 2 * np.arctan(np.sqrt(k2) * dt / 2)) < 1e-12
    e_nm1 = (np.cos(theta) * v)[None]
    e_n = v[None].copy()
    zero = np.zeros_like(e_n)
    worst = 0.0
    for n in range(1, 51):
        e_np1 = o.step(e_n, e_nm1, zero, zero)
        worst = max(worst, np.abs(e_np1[0] - np.cos(n * theta) * v).max())
        e_nm1, e_n = e_n, e_np1
    assert worst < 1e-12 * np.abs(v).max() * 10


def test_energy_invariant_after_source_stops():
    o = _oracle(4, dt=0.1, seed=5)
    N, m = 40, 10
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, 0.1, 0.5, 0.2, seed=3, nrhs=2)
    J[m:] = 0.0
    E = o.run(J)
    H = np.array([o.energy(E[n + 1], E[n]) for n in range(m + 1, N)])
    assert np.ptp(H, axis=0).max() <= 1e-12 * H.max()
    assert H.max() > 0


@pytest.mark.parametrize("grade", [1.0, 1.5])
def test_gauss_law_exact(grade):
    o = _oracle(4, dt=0.05, seed=9, grade=grade)
    N = 30
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, 0.05, 0.75, 0.2, seed=0, nrhs=2)
    E = o.run(J)
    q = o.charge_history(J)
    worst = max(np.abs(o.gauss_residual(E[n], q[n])).max() for n in range(N + 1))
    assert np.abs(q).max() > 1e-3
    assert worst <= 1e-12 * np.abs(q).max()


def test_gauss_law_detects_wrong_source_form():
    """The same check fails for a source sampled without the time-integrated
    current (J^{n+1/2} + J^{n-1/2} instead of the difference)."""
    o = _oracle(3, dt=0.05)
    N = 10
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, 0.05, 0.25, 0.1, seed=0)
    Jr = o.d.restrict(J)
    e = np.zeros((N + 1, 1, o.d.n_int)); em1 = np.zeros((1, o.d.n_int)); Jp = np.zeros((1, o.d.n_int))
    for n in range(N):
        b = (o.B1 @ e[n].T).T - (o.A @ em1.T).T - o.dt * (Jr[n] + Jp)
        e[n + 1] = o.solve(b); em1 = e[n]; Jp = Jr[n]
    q = o.charge_history(J)
    res = np.abs(o.gauss_residual(o.d.extend(e[N]), q[N])).max()
    assert res > 1e-3 * np.abs(q).max()


def test_direct_solve_matches_dense():
    o = _oracle(3, dt=0.07, seed=2)
    b = np.random.default_rng(1).standard_normal((3, o.d.n_int))
    x = o.solve(b)
    xd = np.linalg.solve(o.A.toarray(), b.T).T
    np.testing.assert_allclose(x, xd, rtol=0, atol=1e-12 * np.abs(xd).max())
    r = (o.A @ x.T).T - b
    assert np.linalg.norm(r) <= 1e-14 * np.linalg.norm(b) * 10


def test_relative_residual_property():
    o = _oracle(3, dt=0.05, seed=4)
    J = dense_random_source(o.d.n_e, ~o.d.pec, 5, 0.05, 0.1, 0.05, seed=1, nrhs=2)
    E = o.run(J)
    res = o.relative_residual(E[3], E[2], E[1], J[2], J[1])
    assert res.max() < 1e-14
    bad = E[3].copy(); bad[:, o.d.interior[5]] += 1e-6
    assert o.relative_residual(bad, E[2], E[1], J[2], J[1]).max() > 1e-9


def _loss_setup(seed=0):
    o = _oracle(3, dt=0.05, seed=seed)
    N = 8
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, 0.05, 0.2, 0.08, seed=7)
    probes = o.d.interior[np.random.default_rng(4).choice(o.d.n_int, 10, replace=False)]
    return o, J, probes


def test_adjoint_dot_product():
    """e^N is linear in J:  <ebar, e^N(dJ)> = <Jbar(ebar), dJ>."""
    o, J, _ = _loss_setup()
    rng = np.random.default_rng(12)
    dJ = rng.standard_normal(J.shape); dJ[..., o.d.pec] = 0.0
    E = o.run(dJ)
    ebar = rng.standard_normal(E[-1].shape); ebar[..., o.d.pec] = 0.0
    Jbar, _ = o.adjoint(dJ, E, ebar)
    lhs = np.sum(ebar * E[-1])
    rhs = np.sum(Jbar * dJ)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300)


def test_adjoint_central_differences():
    """Gradient of L = sum_probes (e^N)^2 in eps and J vs central FD (h=1e-6,
    direct solves, so the FD noise is at rounding level)."""
    o, J, probes = _loss_setup()
    c, t, _ = cube_mesh(3)
    eps0 = o.d.eps.copy()

    def loss(eps, Jx):
        oo = NewmarkOracle(c, t, eps=eps, dt=o.dt, beta=o.beta)
        E = oo.run(Jx)
        return np.sum(E[-1][:, probes] ** 2), E

    L0, E = loss(eps0, J)
    ebar = np.zeros_like(E[-1]); ebar[:, probes] = 2 * E[-1][:, probes]
    Jbar, eps_bar = o.adjoint(J, E, ebar)
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(3):
        de = rng.standard_normal(len(eps0))
        dJ = rng.standard_normal(J.shape); dJ[..., o.d.pec] = 0.0
        nrm = np.sqrt(np.sum(de ** 2) + np.sum(dJ ** 2)); de /= nrm; dJ /= nrm
        fd = (loss(eps0 + h * de, J + h * dJ)[0] - loss(eps0 - h * de, J - h * dJ)[0]) / (2 * h)
        ad = np.dot(eps_bar, de) + np.sum(Jbar * dJ)
        assert abs(fd - ad) <= 1e-6 * max(abs(fd), abs(ad)), (fd, ad)


# ---- the iterative path for meshes whose factor does not fit a host --------
def test_mass_lower_bound_is_a_lower_bound():
    """The certified bound min_k eps_k lam_min(T_k) never exceeds the true
    smallest eigenvalue of A (dense eigenvalues, brute force on small
    meshes, uniform and graded, with per-tet eps), and is not vacuous."""
    from oracle.newmark import mass_lower_bound
    for n, grade, seed, dt in ((3, 1.0, None, 0.05), (3, 1.5, 4, 0.1), (4, 1.0, 2, 0.02)):
        o = _oracle(n, dt=dt, seed=seed, grade=grade)
        lo = mass_lower_bound(o.d)
        lam = np.linalg.eigvalsh(o.A.toarray())[0]
        tmin = np.linalg.eigvalsh(o.d.T.toarray())[0]
        assert 0 < lo <= tmin <= lam
        assert lo >= 1e-3 * lam


@pytest.mark.parametrize("n,grade,seed", [(8, 1.0, None), (10, 1.5, 3)])
def test_pcg_matches_direct_over_steps(n, grade, seed):
    """Jacobi PCG (tolerance 1e-13) against the nested-dissection SuperLU
    solve over 12 Newmark steps with 3 right-hand sides, and its certified
    error bound against the actual error of every solve."""
    c, t, _ = cube_mesh(n, grade)
    eps = None if seed is None else np.random.default_rng(seed).uniform(1, 4, len(t))
    od = NewmarkOracle(c, t, eps=eps, dt=0.04, beta=0.25)
    oi = NewmarkOracle(c, t, eps=eps, dt=0.04, beta=0.25, solver="pcg", pcg_tol=1e-13)
    N = 12
    J = dense_random_source(od.d.n_e, ~od.d.pec, N, 0.04, 0.2, 0.08, seed=11, nrhs=3)
    Ed = od.run(J)
    Ei = oi.run(J)
    for k in range(1, N + 1):
        err = np.linalg.norm(Ei[k] - Ed[k], axis=1) / np.linalg.norm(Ed[k], axis=1)
        assert err.max() <= 1e-11, (k, err)
    # the bound of one solve covers its actual error
    rng = np.random.default_rng(2)
    b = rng.standard_normal((3, od.d.n_int))
    xd = od.solve(b)
    xi = oi.solve(b)
    actual = (np.linalg.norm(xi - xd, axis=1) / np.linalg.norm(xd, axis=1)).max()
    it, rel, bound = oi.solve_log[-1]
    assert rel <= 1e-13 and actual <= bound <= 1e-9, (actual, bound)


def test_pcg_bound_reports_a_loose_solve():
    """A solve stopped early reports a residual and a bound that cover the
    error it really has (the bound is what the full-size fixtures rely on)."""
    from oracle.newmark import pcg
    o = _oracle(6, dt=0.05, seed=1)
    oi = NewmarkOracle(o.d.coords, o.d.tets, eps=o.d.eps, dt=0.05, solver="pcg", pcg_tol=1e-4)
    b = np.random.default_rng(3).standard_normal((2, o.d.n_int))
    xd = o.solve(b)
    xi = oi.solve(b)
    actual = (np.linalg.norm(xi - xd, axis=1) / np.linalg.norm(xd, axis=1)).max()
    it, rel, bound = oi.solve_log[-1]
    assert 1e-10 < actual <= bound
    x, _, rel2 = pcg(o.A, b.T, tol=1e-4)
    assert rel2.max() <= 1e-4


# ---- extended precision for finite differences --------------------------------
def test_inverse_by_cofactors_matches_lapack():
    from oracle.fem import _inv3
    D = np.random.default_rng(0).standard_normal((50, 3, 3))
    inv, det = _inv3(D)
    np.testing.assert_allclose(inv, np.linalg.inv(D), rtol=0, atol=1e-12 * np.abs(np.linalg.inv(D)).max())
    np.testing.assert_allclose(det, np.linalg.det(D), rtol=1e-12)


def test_extended_forward_matches_fp64_and_sharpens_fd():
    """The extended-precision recurrence (80-bit assembly and residuals,
    FP64 factor refined) solves the same equations as the FP64 direct path
    (agreement to FP64 rounding), and its central differences at h = 1e-6
    match the FP64 adjoint far more tightly than FP64 forwards can, whose
    rounding floor is about 1e-16 L / h."""
    o, J, probes = _loss_setup()
    c, t, _ = cube_mesh(3)
    eps0 = o.d.eps.copy()
    E = o.run(J)
    ox = NewmarkOracle(c, t, eps=eps0, dt=o.dt, beta=o.beta, solver="extended")
    Ex = ox.run(J)
    assert Ex.dtype == np.longdouble
    err = np.abs(Ex.astype(np.float64) - E).max() / np.abs(E).max()
    assert err <= 1e-13, err
    ebar = np.zeros_like(E[-1]); ebar[:, probes] = 2 * E[-1][:, probes]
    Jbar, eps_bar = o.adjoint(J, E, ebar)
    rng = np.random.default_rng(8)
    h = np.longdouble(1e-6)

    def loss(eps, Jx):
        oo = NewmarkOracle(c, t, eps=eps, dt=o.dt, beta=o.beta, solver="extended")
        return np.sum(oo.run(Jx)[-1][:, probes] ** 2)

    for _ in range(3):
        de = rng.standard_normal(len(eps0))
        dJ = rng.standard_normal(J.shape); dJ[..., o.d.pec] = 0.0
        nrm = np.sqrt(np.sum(de ** 2) + np.sum(dJ ** 2)); de /= nrm; dJ /= nrm
        e_l, J_l = eps0.astype(np.longdouble), J.astype(np.longdouble)
        fd = float((loss(e_l + h * de, J_l + h * dJ) - loss(e_l - h * de, J_l - h * dJ)) / (2 * h))
        ad = np.dot(eps_bar, de) + np.sum(Jbar * dJ)
        assert abs(fd - ad) <= 1e-9 * max(abs(fd), abs(ad)), (fd, ad)
