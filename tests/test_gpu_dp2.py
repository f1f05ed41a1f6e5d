"""GPU parity of the Robin dual-primal variant (Sec. III-B adapted to the
edge-only system: one multiplier per interface side, transmission condition
lam_i + lam_j + 2 alpha M_T x_j = 0, restarted GMRES) against the FP64 oracle,
the monolithic direct solve.  At a converged fixed point the Robin terms
cancel (the condition on both sides forces equal interface values and
opposite fluxes), so the decomposed fields equal the monolithic ones; the
bar is the same as for the first variant: rel. L2 <= 1e-10 in FP64 and
<= 1e-8 with FP32 factors and FP64 refinement."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.newmark import NewmarkOracle
from workloads.mesh import cube_mesh, jittered_cube_mesh
from workloads.partition import box_partition, rcb_partition
from workloads.sources import dense_random_source

pytestmark = pytest.mark.gpu


def _solver(*a, **k):
    from paper_2204_13254_amd.solver import DDSolver
    return DDSolver(*a, method="dp2", **k)


def relerr(x, y):
    num = np.linalg.norm(np.asarray(x) - np.asarray(y), axis=-1)
    den = np.linalg.norm(np.asarray(y), axis=-1)
    return np.where(den > 0, num / np.where(den > 0, den, 1), num)


@pytest.mark.parametrize("n,parts,eps_seed,nrhs,alpha", [
    (4, 2, None, 1, 0.0),
    (6, 3, 7, 2, 0.0),
    (8, ("rcb", 3, 1), 3, 3, 0.0),
    (6, 2, None, 1, 0.5),
])
def test_single_solve_fp64(n, parts, eps_seed, nrhs, alpha):
    c, t, _ = cube_mesh(n)
    p = rcb_partition(n, parts[1], parts[2]) if isinstance(parts, tuple) else box_partition(n, parts)
    eps = np.ones(len(t)) if eps_seed is None else np.random.default_rng(eps_seed).uniform(1, 4, len(t))
    print(f"case n={n} parts={parts} nrhs={nrhs} alpha={alpha}", flush=True)
    s = _solver(c, t, p, eps, dt=0.05, nrhs=nrhs, cg_tol=1e-13, cg_max_iter=400, robin_alpha=alpha)
    o = NewmarkOracle(c, t, eps=eps, dt=0.05)
    b = np.random.default_rng(1).standard_normal((nrhs, o.d.n_e))
    b[:, o.d.pec] = 0.0
    x = s.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    st = s.last_stats()
    print("gmres iterations", st["cg_iters"], "relres", st["cg_relres"], flush=True)
    xr = o.d.extend(o.solve(o.d.restrict(b)))
    err = relerr(x, xr)
    assert err.max() <= 1e-10, err
    assert np.all(x[:, o.d.pec] == 0.0)


def _run(s, J):
    N, nrhs, ne = J.shape
    Jd = torch.tensor(J, device="cuda")
    zero = torch.zeros((nrhs, ne), dtype=torch.float64, device="cuda")
    E = [zero, zero.clone()]
    Jprev = zero
    its = []
    for k in range(N):
        E.append(s.step(Jd[k], Jprev, E[-1], E[-2], stats=True))
        its.append(s.last_stats()["solve_iters"][:1 + s.last_stats()["refine_sweeps"]])
        Jprev = Jd[k]
    return torch.stack(E[1:]).cpu().numpy(), its


@pytest.mark.parametrize("prec,tol,nrhs", [("fp64", 1e-10, 2), ("fp32_refine", 1e-8, 3)])
def test_newmark_steps_jittered(prec, tol, nrhs):
    """Jittered 6^3 mesh (unstructured), 8 subdomains, random eps, 8 steps."""
    n, dt = 6, 0.04
    c, t, _ = jittered_cube_mesh(n, 0.15, 3)
    p = box_partition(n, 2)
    eps = np.random.default_rng(5).uniform(1, 3, len(t))
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    J = dense_random_source(o.d.n_e, ~o.d.pec, 8, dt, 0.12, 0.04, seed=8, nrhs=nrhs)
    s = _solver(c, t, p, eps, dt=dt, nrhs=nrhs, precision=prec,
                cg_tol=1e-12 if prec == "fp64" else 1e-6, refine_tol=1e-12, cg_max_iter=400)
    E, its = _run(s, J)
    Eo = o.run(J)
    err = relerr(E[1:], Eo[1:])
    print(prec, "max rel err", err.max(), "iterations", its, flush=True)
    assert err.max() <= tol


def test_same_answer_as_first_variant():
    """Both decompositions solve the same monolithic system."""
    from paper_2204_13254_amd.solver import DDSolver
    n = 8
    c, t, _ = cube_mesh(n)
    p = box_partition(n, 2)
    eps = np.ones(len(t))
    s1 = DDSolver(c, t, p, eps, dt=0.05, nrhs=2, cg_tol=1e-13)
    s2 = _solver(c, t, p, eps, dt=0.05, nrhs=2, cg_tol=1e-13, cg_max_iter=400)
    bb = np.random.default_rng(4).standard_normal((2, s1.n_edges))
    e, pec = s1.edges()
    bb[:, pec.astype(bool)] = 0.0
    x1 = s1.solve(torch.tensor(bb, device="cuda")).cpu().numpy()
    x2 = s2.solve(torch.tensor(bb, device="cuda")).cpu().numpy()
    assert relerr(x2, x1).max() <= 1e-10


@pytest.mark.parametrize("method", ["dp1", "dp2"])
def test_one_subdomain_and_zero_rhs(method):
    """Degenerate decompositions: one subdomain (no multipliers, no corners:
    the stored inverse is the whole solve) and a zero right-hand side."""
    from paper_2204_13254_amd.solver import DDSolver
    n = 4
    c, t, _ = cube_mesh(n)
    eps = np.random.default_rng(2).uniform(1, 2, len(t))
    o = NewmarkOracle(c, t, eps=eps, dt=0.05)
    b = np.random.default_rng(5).standard_normal((2, o.d.n_e))
    b[:, o.d.pec] = 0.0
    for parts in (1, 2):
        s = DDSolver(c, t, box_partition(n, parts), eps, dt=0.05, nrhs=2, cg_tol=1e-13, cg_max_iter=400,
                     method=method)
        x = s.solve(torch.tensor(b, device="cuda")).cpu().numpy()
        assert relerr(x, o.d.extend(o.solve(o.d.restrict(b)))).max() <= 1e-10
        z = s.solve(torch.zeros((2, o.d.n_e), dtype=torch.float64, device="cuda")).cpu().numpy()
        assert np.all(z == 0.0)


def test_dp2_32_rhs_fp32_refine():
    """The widest right-hand-side block with the Robin variant."""
    n, dt, nrhs = 6, 0.04, 32
    c, t, _ = cube_mesh(n)
    p = rcb_partition(n, 3, 2)
    eps = np.ones(len(t))
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    J = dense_random_source(o.d.n_e, ~o.d.pec, 3, dt, 0.06, 0.03, seed=12, nrhs=nrhs)
    s = _solver(c, t, p, eps, dt=dt, nrhs=nrhs, precision="fp32_refine", cg_tol=1e-6, refine_tol=1e-12,
                cg_max_iter=400)
    E, its = _run(s, J)
    err = relerr(E[1:], o.run(J)[1:])
    print("32 rhs max rel err", err.max(), "iterations", its, flush=True)
    assert err.max() <= 1e-8


def test_dp2_adjoint_step_matches_first_variant():
    """The reverse step reuses the decomposed solve (A is symmetric); both
    variants give the same adjoint quantities."""
    from paper_2204_13254_amd.solver import DDSolver
    n, dt = 5, 0.05
    c, t, _ = cube_mesh(n)
    p = box_partition(n, 2)
    eps = np.random.default_rng(6).uniform(1, 3, len(t))
    rng = np.random.default_rng(9)
    out = {}
    for method in ("dp1", "dp2"):
        s = DDSolver(c, t, p, eps, dt=dt, cg_tol=1e-13, cg_max_iter=400, method=method)
        ne = s.n_edges
        _, pec = s.edges()
        vals = rng.standard_normal((4, 1, ne)) if method == "dp1" else vals
        v = vals.copy()
        v[:, :, pec.astype(bool)] = 0.0
        d = [torch.tensor(x, device="cuda") for x in v]
        eb_n = torch.zeros((1, ne), dtype=torch.float64, device="cuda")
        eb_m = torch.zeros((1, ne), dtype=torch.float64, device="cuda")
        epsbar = torch.zeros(len(t), dtype=torch.float64, device="cuda")
        g = s.adjoint_step(d[0], eb_n, eb_m, d[1], d[2], d[3], epsbar)
        out[method] = [x.cpu().numpy() for x in (g, eb_n, eb_m, epsbar)]
    for a, b in zip(out["dp2"], out["dp1"]):
        assert relerr(a.reshape(1, -1), b.reshape(1, -1)).max() <= 1e-10
