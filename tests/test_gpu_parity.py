"""GPU parity of the decomposed solve (HIP library through the C ABI) against
the FP64 oracle (the monolithic direct solve), element by element.

The decomposition is exact (Sec. IV-A: decomposed and monolithic fields agree
to near machine precision), so the tolerance is set by the interface CG and
refinement tolerances: rel. L2 <= 1e-10 in FP64 and <= 1e-8 for FP32 factors
with FP64 refinement, at every step and for every right-hand side."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.newmark import NewmarkOracle
from workloads.configs import workload
from workloads.mesh import centred_cube_mesh, cube_mesh
from workloads.partition import box_partition, rcb_partition
from workloads.sources import dense_random_source

pytestmark = pytest.mark.gpu


def _solver(*a, **k):
    from paper_2204_13254_amd.solver import DDSolver
    return DDSolver(*a, **k)


def relerr(x, y, mask=None):
    x = np.asarray(x); y = np.asarray(y)
    num = np.linalg.norm(x - y, axis=-1)
    den = np.linalg.norm(y, axis=-1)
    return np.where(den > 0, num / np.where(den > 0, den, 1), num)


def _case(n, parts, grade=1.0, eps_seed=None, dt=0.05):
    c, t, _ = cube_mesh(n, grade)
    if isinstance(parts, tuple) and parts[0] == "rcb":
        p = rcb_partition(n, parts[1], parts[2])
    else:
        p = box_partition(n, parts)
    eps = np.ones(len(t)) if eps_seed is None else np.random.default_rng(eps_seed).uniform(1, 4, len(t))
    return c, t, p, eps


def test_edges_match_oracle():
    c, t, p, eps = _case(4, 2)
    s = _solver(c, t, p, eps, dt=0.05, factor=False)
    e, pec = s.edges()
    o = NewmarkOracle(c, t, dt=0.05, factor=False)
    assert np.array_equal(e, o.d.edges)
    assert np.array_equal(pec, o.d.pec)


@pytest.mark.parametrize("n,parts,grade,eps_seed,nrhs", [
    (4, 2, 1.0, None, 1),
    (6, 3, 1.0, 7, 2),
    (8, ("rcb", 3, 1), 1.5, 3, 3),
    (9, (2, 3, 1), 1.0, 5, 1),
])
def test_single_solve_fp64(n, parts, grade, eps_seed, nrhs):
    c, t, p, eps = _case(n, parts, grade, eps_seed)
    print(f"case n={n} parts={parts} nrhs={nrhs}", flush=True)
    s = _solver(c, t, p, eps, dt=0.05, nrhs=nrhs, cg_tol=1e-13)
    o = NewmarkOracle(c, t, eps=eps, dt=0.05)
    b = np.random.default_rng(1).standard_normal((nrhs, o.d.n_e))
    b[:, o.d.pec] = 0.0
    x = s.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    xr = o.d.extend(o.solve(o.d.restrict(b)))
    err = relerr(x, xr)
    assert err.max() <= 1e-10, err
    assert np.all(x[:, o.d.pec] == 0.0)


def _run_dd(s, J):
    N, nrhs, ne = J.shape
    Jd = torch.tensor(J, device="cuda")
    zero = torch.zeros((nrhs, ne), dtype=torch.float64, device="cuda")
    E = [zero, zero.clone()]   # e^{-1}, e^0
    Jprev = zero
    iters = []
    for n in range(N):
        E.append(s.step(Jd[n], Jprev, E[-1], E[-2], stats=True))
        iters.append(s.last_stats()["cg_iters"])
        Jprev = Jd[n]
    return torch.stack(E[1:]).cpu().numpy(), iters


def test_small_workload_fp64_every_step():
    """8^3 cavity, 2x2x2 boxes, 10 steps, CG tol 1e-12: <= 1e-10 per step."""
    w = workload(1)
    c, t = w.mesh(); p = w.partition()
    J = w.sources(t, c)
    s = _solver(c, t, p, w.eps(len(t)), dt=w.dt, beta=w.beta, cg_tol=w.cg_tol)
    E, iters = _run_dd(s, J)
    o = NewmarkOracle(c, t, dt=w.dt, beta=w.beta)
    Eo = o.run(J)
    err = relerr(E[1:], Eo[1:])
    print("max rel err", err.max(), "iters", iters, flush=True)
    assert err.max() <= 1e-10


@pytest.mark.parametrize("prec,tol,nrhs", [("fp64", 1e-10, 2), ("fp32_refine", 1e-8, 4)])
def test_uneven_graded_multi_rhs(prec, tol, nrhs):
    """Graded 10^3 mesh, 16 uneven recursive-bisection subdomains, random
    eps, several right-hand sides, 12 steps."""
    c, t, p, eps = _case(10, ("rcb", 4, 2), grade=1.5, eps_seed=11)
    dt = 0.03
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    J = dense_random_source(o.d.n_e, ~o.d.pec, 12, dt, 0.18, 0.05, seed=21, nrhs=nrhs)
    s = _solver(c, t, p, eps, dt=dt, nrhs=nrhs, precision=prec,
                cg_tol=1e-12 if prec == "fp64" else 1e-6, refine_tol=1e-12)
    E, iters = _run_dd(s, J)
    Eo = o.run(J)
    err = relerr(E[1:], Eo[1:])
    print(prec, "max rel err", err.max(), flush=True)
    assert err.max() <= tol


# right-hand-side counts 2, 6, 12 and 24 take the per-thread sparse (T, S)
# product and its cooperative forms with 8, 16 and 32 lanes per row; 8, 16
# and 32 its vector form (two right-hand sides per lane, 4, 8 and 16 lanes
# per row)
@pytest.mark.parametrize("nrhs", [2, 6, 8, 12, 16, 24, 32])
def test_gauss_law_and_energy_match_oracle(nrhs):
    c, t, p, eps = _case(6, 2, eps_seed=4)
    dt = 0.05
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    N = 8
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, dt, 0.2, 0.06, seed=2, nrhs=nrhs)
    J[5:] = 0.0
    s = _solver(c, t, p, eps, dt=dt, nrhs=nrhs, cg_tol=1e-13)
    E, _ = _run_dd(s, J)
    q = torch.zeros((nrhs, s.n_vertices), dtype=torch.float64, device="cuda")
    Jd = torch.tensor(J, device="cuda")
    qo = o.charge_history(J)
    for n in range(N):
        s.charge_update(Jd[n], q)
        res = s.gauss_residual(torch.tensor(E[n + 1], device="cuda"), q)
        assert res.max() <= 1e-9 * max(1e-30, np.abs(qo[n + 1]).max())
    H = s.energy(torch.tensor(E[-1], device="cuda"), torch.tensor(E[-2], device="cuda"))
    Ho = o.energy(E[-1], E[-2])
    np.testing.assert_allclose(H, Ho, rtol=1e-12)


@pytest.mark.parametrize("nrhs", [1, 6, 12, 24])
def test_adjoint_step_matches_oracle(nrhs):
    c, t, p, eps = _case(5, 2, eps_seed=6)
    dt = 0.05
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    N = 6
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, dt, 0.15, 0.05, seed=8, nrhs=nrhs)
    E = o.run(J)
    rng = np.random.default_rng(3)
    ebar = rng.standard_normal(E[-1].shape); ebar[:, o.d.pec] = 0.0
    Jbar_o, epsbar_o = o.adjoint(J, E, ebar)
    s = _solver(c, t, p, eps, dt=dt, nrhs=nrhs, cg_tol=1e-13)
    dev = lambda a: torch.tensor(a, device="cuda")
    eb = [torch.zeros((nrhs, o.d.n_e), dtype=torch.float64, device="cuda") for _ in range(N + 1)]
    eb[N] = dev(ebar)
    epsbar = torch.zeros(len(t), dtype=torch.float64, device="cuda")
    # the library accumulates the current adjoints itself
    Jbar = torch.zeros((N, nrhs, o.d.n_e), dtype=torch.float64, device="cuda")
    for n in range(N - 1, -1, -1):
        s.adjoint_step(eb[n + 1], eb[n], eb[n - 1] if n >= 1 else None, dev(E[n + 1]), dev(E[n]),
                       dev(E[n - 1]) if n >= 1 else None, epsbar,
                       Jbar_half=Jbar[n], Jbar_prev_half=Jbar[n - 1] if n >= 1 else None)
    assert relerr(Jbar.cpu().numpy().reshape(-1), Jbar_o.reshape(-1)) <= 1e-9
    assert relerr(epsbar.cpu().numpy(), epsbar_o) <= 1e-9


@pytest.mark.parametrize("prec,nrhs", [("fp64", 3), ("fp32_refine", 16)])
def test_step_diagnostics_match_oracle(prec, nrhs):
    """dd_step's per-step checks (DD_DIAG_GAUSS | DD_DIAG_ENERGY): the
    accumulated nodal charge, the Gauss residual max |G^T T e^{n+1} +
    q^{n+1}| and the energy H^{n+1/2} against the oracle's own evaluation of
    the same quantities from the oracle's fields, at every step (Sec. IV-B:
    charge conservation)."""
    c, t, p, eps = _case(6, ("rcb", 3, 2), grade=1.5, eps_seed=3)
    dt = 0.05
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    N = 6
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, dt, 0.1, 0.04, seed=5, nrhs=nrhs)
    Eo = o.run(J)
    qo = o.charge_history(J)
    s = _solver(c, t, p, eps, dt=dt, nrhs=nrhs, precision=prec, diagnostics=3,
                cg_tol=1e-12 if prec == "fp64" else 1e-6)
    Jd = torch.tensor(J, device="cuda")
    z = s.new_field()
    E = [z, z.clone()]
    for n in range(N):
        E.append(s.step(Jd[n], Jd[n - 1] if n else z, E[-1], E[-2], stats=True))
        st = s.last_stats()
        assert st["diagnostics"] == 3
        qmax = np.abs(qo[n + 1]).max(axis=1)
        np.testing.assert_allclose(st["charge_max"], qmax, rtol=1e-12)
        # the oracle's residual is at rounding level; the library's is bounded
        # by its solve tolerance times the charge scale
        assert np.all(np.array(st["gauss_residual"]) <= 1e-9 * qmax), (n, st["gauss_residual"], qmax)
        Ho = o.energy(Eo[n + 1], Eo[n])
        np.testing.assert_allclose(st["energy"], Ho, rtol=1e-8)
    # dd_set_charge: a restart from zero charge at a nonzero field breaks the law
    s.set_charge(None)
    s.step(Jd[0], z, E[-1], E[-2], stats=True)
    assert max(s.last_stats()["gauss_residual"]) > 1e-6 * np.abs(qo[1:]).max()


def test_nonfinite_load_and_not_spd_reported():
    """A NaN in the current is reported as DD_ERR_NONFINITE (naming the RHS)
    instead of being iterated on.  A permittivity of 1e60 in subdomain 3
    overflows that subdomain's FP32 matrix (valid input, not representable
    in the factor precision): the factor meets non-finite pivots there and
    reports DD_ERR_NOT_SPD naming subdomain 3, after which steps are
    refused until a factorisation succeeds."""
    from paper_2204_13254_amd import DDError
    c, t, p, eps = _case(4, 2)
    s = _solver(c, t, p, eps, dt=0.05, nrhs=2)
    z = s.new_field()
    J = torch.zeros_like(z)
    _, pec = s.edges()
    J[1, int(np.flatnonzero(~pec)[5])] = float("nan")     # an unknown (conductor entries are ignored)
    with pytest.raises(DDError, match="DD_ERR_NONFINITE.*right-hand side 1"):
        s.step(J, z, z, z, z)
    s.step(z, z, z, z, z)                  # the context stays usable
    big = np.where(p == 3, 1e60, 1.0)
    s32 = _solver(c, t, p, big, dt=0.05, precision="fp32_refine", factor=False)
    with pytest.raises(DDError, match="DD_ERR_NOT_SPD.*subdomain 3$"):
        s32.factor()
    with pytest.raises(DDError, match="DD_ERR_STATE"):
        s32.step(z[:1], z[:1], z[:1], z[:1], z[:1].clone())
    s32.set_eps(eps)
    s32.factor()
    s32.step(z[:1], z[:1], z[:1], z[:1], z[:1].clone())


def test_set_eps_from_device_matches_host():
    """dd_set_eps with a device array gives the same factors (bit-identical
    fields) as the host array, and rejects a non-positive entry."""
    from paper_2204_13254_amd import DDError
    c, t, p, eps = _case(5, 2, eps_seed=1)
    dt = 0.05
    o = NewmarkOracle(c, t, dt=dt, factor=False)
    J = dense_random_source(o.d.n_e, ~o.d.pec, 3, dt, 0.05, 0.03, seed=2, nrhs=1)
    out = []
    for on_dev in (False, True):
        s = _solver(c, t, p, np.ones(len(t)), dt=dt)
        s.set_eps(torch.tensor(eps, device="cuda") if on_dev else eps)
        s.factor()
        out.append(_run_dd(s, J)[0])
    assert np.array_equal(out[0], out[1])
    bad = torch.tensor(eps, device="cuda")
    bad[7] = -1.0
    with pytest.raises(DDError, match="DD_ERR_ARG"):
        s.set_eps(bad)


def test_errors_reported():
    from paper_2204_13254_amd import DDError
    c, t, p, eps = _case(4, 2)
    s = _solver(c, t, p, eps, dt=0.05, factor=False)
    z = s.new_field()
    with pytest.raises(DDError, match="DD_ERR_STATE"):
        s.step(z, z, z, z, z)
    s2 = _solver(c, t, p, eps, dt=0.05, cg_max_iter=1, cg_tol=1e-14, check_every=1)
    b = torch.randn((1, s2.n_edges), dtype=torch.float64, device="cuda")
    with pytest.raises(DDError, match="DD_ERR_NO_CONVERGENCE"):
        s2.solve(b)
    # the context stays usable
    s2.solve(torch.zeros_like(b))
    with pytest.raises(DDError, match="DD_ERR_ARG"):
        _solver(c, t, p, -eps, dt=0.05)
    with pytest.raises(DDError, match="DD_ERR_PARTITION"):
        _solver(c, t, p + 1, eps, dt=0.05)


@pytest.mark.parametrize("prec,nrhs,tol", [("fp64", 12, 1e-10), ("fp32_refine", 16, 1e-8),
                                           ("fp32_refine", 20, 1e-8), ("fp64", 5, 1e-10),
                                           ("fp64", 32, 1e-10)])
def test_rhs_block_paths(prec, nrhs, tol):
    """Every right-hand-side block width of the tile products (vector FMA
    for <= 8, MFMA 16x16x4 for 9..32) and of the symmetric interface product
    (MFMA, one or two 16-wide RHS blocks) on an uneven partition with
    corners."""
    c, t, p, eps = _case(8, ("rcb", 3, 5), grade=1.5, eps_seed=13)
    dt = 0.04
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    J = dense_random_source(o.d.n_e, ~o.d.pec, 4, dt, 0.08, 0.03, seed=31, nrhs=nrhs)
    s = _solver(c, t, p, eps, dt=dt, nrhs=nrhs, precision=prec,
                cg_tol=1e-12 if prec == "fp64" else 1e-6)
    E, _ = _run_dd(s, J)
    err = relerr(E[1:], o.run(J)[1:])
    print(prec, nrhs, "max rel err", err.max(), flush=True)
    assert err.max() <= tol


@pytest.mark.parametrize("prec,nrhs,tol", [("fp64", 1, 1e-10), ("fp32_refine", 16, 1e-8)])
def test_preconditioner_on_off(prec, nrhs, tol):
    """The interface CG with and without the lumped preconditioner reaches
    the oracle's fields at every step; the preconditioned one in fewer
    iterations."""
    c, t, p, eps = _case(8, ("rcb", 3, 5), grade=1.5, eps_seed=13)
    dt = 0.04
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    J = dense_random_source(o.d.n_e, ~o.d.pec, 4, dt, 0.08, 0.03, seed=37, nrhs=nrhs)
    Eo = o.run(J)
    its = {}
    for pc in (0, 1):
        s = _solver(c, t, p, eps, dt=dt, nrhs=nrhs, precision=prec,
                    cg_tol=1e-12 if prec == "fp64" else 1e-6, precond=pc)
        E, iters = _run_dd(s, J)
        err = relerr(E[1:], Eo[1:])
        print(prec, "precond", pc, "max rel err", err.max(), "iterations", iters, flush=True)
        assert err.max() <= tol
        its[pc] = sum(sum(x) if isinstance(x, (list, tuple)) else x for x in iters)
    assert its[1] < its[0]


def test_graph_replay_matches_eager():
    """The CG iteration blocks replayed from a captured HIP graph (on a
    non-default stream, with the eager pre-solve / recovery / refinement work
    and host synchronisations between replays) give bit-identical fields to
    eager launches at every step (all reductions have a fixed order)."""
    c, t, p, eps = _case(8, ("rcb", 3, 5), grade=1.5, eps_seed=13)
    dt = 0.04
    o = NewmarkOracle(c, t, eps=eps, dt=dt, factor=False)
    J = dense_random_source(o.d.n_e, ~o.d.pec, 6, dt, 0.1, 0.03, seed=41, nrhs=16)
    out = {}
    for g in (False, True):
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            s = _solver(c, t, p, eps, dt=dt, nrhs=16, precision="fp32_refine", cg_tol=1e-6,
                        use_graph=g, check_every=3, stream=st)
            E, iters = _run_dd(s, J)
        st.synchronize()
        out[g] = (E, iters)
    assert np.array_equal(out[True][0], out[False][0])
    assert out[True][1] == out[False][1]


def test_captured_step_adapts_its_budget():
    """The refined step as one captured graph: sized by the previous step's
    CG iterations and sweeps, so a step that needs more than the capture
    holds (here: zero sources first, capture sized for 1 iteration and no
    sweep, then a pulse) finishes its refinement eagerly and re-sizes the
    next capture.  Every step against the oracle; the captured steps of a
    steady run give the same fields bit for bit as eager launches."""
    c, t, p, eps = _case(8, ("rcb", 3, 5), grade=1.5, eps_seed=13)
    dt = 0.04
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    N = 9
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, dt, 0.2, 0.05, seed=43, nrhs=16)
    J[:3] = 0.0
    Eo = o.run(J)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = _solver(c, t, p, eps, dt=dt, nrhs=16, precision="fp32_refine", cg_tol=1e-6, use_graph=True,
                    stream=st)
        E, iters = _run_dd(s, J)
    st.synchronize()
    for k in range(4, N + 1):
        assert relerr(E[k], Eo[k]).max() <= 1e-8, k
    assert np.abs(E[:4]).max() == 0.0
    # steady run: captured (use_graph) and eager steps agree bit for bit
    J2 = dense_random_source(o.d.n_e, ~o.d.pec, 6, dt, 0.1, 0.05, seed=47, nrhs=16)
    out = {}
    for g in (False, True):
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            s = _solver(c, t, p, eps, dt=dt, nrhs=16, precision="fp32_refine", cg_tol=1e-6, use_graph=g,
                        stream=st)
            out[g] = _run_dd(s, J2)
        st.synchronize()
    assert np.array_equal(out[True][0], out[False][0])
    assert out[True][1] == out[False][1]


@pytest.mark.parametrize("prec,nrhs,tol", [("fp64", 3, 1e-10), ("fp64", 6, 1e-10),
                                           ("fp32_refine", 16, 1e-8), ("fp64", 24, 1e-10)])
def test_long_rows_centred_mesh(prec, nrhs, tol):
    """Cubes cut into 12 tetrahedra around their centres: edge-matrix rows of
    up to 25 nonzeros, so the sparse (T, S) products take more than one batch
    of a row's nonzeros, in every lane-group width.  Steps, the energy and the
    Gauss law against the oracle."""
    n = 4
    c, t, _ = centred_cube_mesh(n)
    p = np.repeat(box_partition(n, 2)[::6], 12)
    eps = np.random.default_rng(17).uniform(1, 3, len(t))
    dt = 0.04
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    rows = np.diff((abs(o.d.T) + abs(o.d.S)).tocsr().indptr)
    assert rows.max() > 20
    N = 6
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, dt, 0.1, 0.04, seed=19, nrhs=nrhs)
    Eo = o.run(J)
    s = _solver(c, t, p, eps, dt=dt, nrhs=nrhs, precision=prec,
                cg_tol=1e-13 if prec == "fp64" else 1e-6, refine_tol=1e-12)
    E, _ = _run_dd(s, J)
    for k in range(1, N + 1):
        assert relerr(E[k], Eo[k]).max() <= tol, k
    H = s.energy(torch.tensor(E[-1], device="cuda"), torch.tensor(E[-2], device="cuda"))
    np.testing.assert_allclose(H, o.energy(E[-1], E[-2]), rtol=1e-12)


@pytest.mark.parametrize("parts,prec,nrhs,method,tol", [((2, 1, 1), "fp64", 2, "dp1", 1e-10),
                                                       ((3, 1, 1), "fp32_refine", 16, "dp1", 1e-8),
                                                       ((3, 1, 1), "fp64", 6, "dp2", 1e-10)])
def test_slabs_without_corners(parts, prec, nrhs, method, tol):
    """Slab partitions: every interface edge is shared by two subdomains, so
    there are no corners and no coarse problem; the interface solve runs
    without the corner passes (first variant) or with GMRES (Robin)."""
    from paper_2204_13254_amd.solver import analyze
    n = 6
    c, t, _ = cube_mesh(n)
    p = box_partition(n, parts)
    assert analyze(c, t, p)[1][:, 2].max() == 0
    eps = np.random.default_rng(23).uniform(1, 3, len(t))
    dt = 0.05
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    N = 5
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, dt, 0.12, 0.04, seed=29, nrhs=nrhs)
    Eo = o.run(J)
    s = _solver(c, t, p, eps, dt=dt, nrhs=nrhs, precision=prec, method=method, cg_max_iter=400,
                cg_tol=1e-13 if prec == "fp64" else 1e-6, refine_tol=1e-12)
    E, _ = _run_dd(s, J)
    for k in range(1, N + 1):
        assert relerr(E[k], Eo[k]).max() <= tol, k
