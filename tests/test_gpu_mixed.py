"""GPU parity of the mixed E/B step (dd_step_mixed: B on faces as Whitney
2-forms, trapezoid rule, the eliminated edge system solved by the
decomposition) against the monolithic mixed oracle (oracle/mixed.py), which
solves the full non-symmetric edge + face block system directly.  Bar: rel.
L2 <= 1e-10 (FP64) and <= 1e-8 (FP32 factors + FP64 refinement) for both
fields at every step."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.mixed import MixedOracle
from workloads.mesh import cube_mesh, jittered_cube_mesh
from workloads.partition import box_partition, rcb_partition
from workloads.sources import dense_random_source

pytestmark = pytest.mark.gpu


def relerr(x, y):
    x = np.asarray(x).reshape(len(x), -1)
    y = np.asarray(y).reshape(len(y), -1)
    num = np.linalg.norm(x - y, axis=-1)
    den = np.linalg.norm(y, axis=-1)
    return np.where(den > 0, num / np.where(den > 0, den, 1), num)


def _setup(n, parts, nrhs, prec, method="dp1", jitter=True, seed=3):
    from paper_2204_13254_amd.solver import DDSolver
    c, t, _ = jittered_cube_mesh(n, 0.15, seed) if jitter else cube_mesh(n)
    p = rcb_partition(n, parts[1], parts[2]) if isinstance(parts, tuple) else box_partition(n, parts)
    rng = np.random.default_rng(seed)
    eps = rng.uniform(1, 3, len(t))
    mu = rng.uniform(1, 2, len(t))
    dt = 0.04
    s = DDSolver(c, t, p, eps, mu, dt=dt, beta=0.25, nrhs=nrhs, precision=prec, method=method,
                 cg_tol=1e-13 if prec == "fp64" else 1e-6, refine_tol=1e-12, cg_max_iter=400)
    o = MixedOracle(c, t, eps=eps, mu=mu, dt=dt)
    return s, o, dt


def test_faces_match_oracle():
    s, o, _ = _setup(4, 2, 1, "fp64")
    assert np.array_equal(s.faces(), o.faces)


@pytest.mark.parametrize("n,parts,nrhs,prec,method,tol", [
    (5, 2, 1, "fp64", "dp1", 1e-10),
    (6, ("rcb", 3, 4), 3, "fp32_refine", "dp1", 1e-8),
    (5, 2, 2, "fp64", "dp2", 1e-10),
])
def test_mixed_steps_match_oracle(n, parts, nrhs, prec, method, tol):
    s, o, dt = _setup(n, parts, nrhs, prec, method)
    rng = np.random.default_rng(11)
    N = 8
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, dt, 0.12, 0.04, seed=13, nrhs=nrhs)
    e0 = rng.normal(size=(nrhs, o.d.n_e)); e0[:, o.d.pec] = 0.0
    b0 = np.ascontiguousarray((o.C @ rng.normal(size=(o.d.n_int, nrhs))).T)   # a discrete curl: divergence-free
    Eo, Bo = o.run(J, e0, b0)
    E = torch.tensor(e0, device="cuda")
    B = torch.tensor(b0, device="cuda")
    Jd = torch.tensor(J, device="cuda")
    for k in range(N):
        E, B = s.step_mixed(Jd[k], E, B)
        ee = relerr(E.cpu().numpy(), Eo[k + 1]).max()
        eb = relerr(B.cpu().numpy(), Bo[k + 1]).max()
        print(f"step {k}: e {ee:.2e} b {eb:.2e}", flush=True)
        assert ee <= tol and eb <= tol


def test_mixed_energy_conserved_without_sources():
    s, o, dt = _setup(5, 2, 2, "fp64")
    rng = np.random.default_rng(5)
    e0 = rng.normal(size=(2, o.d.n_e)); e0[:, o.d.pec] = 0.0
    b0 = rng.normal(size=(2, o.n_f))
    E = torch.tensor(e0, device="cuda")
    B = torch.tensor(b0, device="cuda")
    z = torch.zeros_like(E)
    H0 = o.energy(e0, b0)
    for _ in range(6):
        E, B = s.step_mixed(z, E, B)
    H = o.energy(E.cpu().numpy(), B.cpu().numpy())
    assert np.abs(H - H0).max() <= 1e-10 * H0.max()


def test_mixed_needs_quarter_beta():
    from paper_2204_13254_amd import DDError
    from paper_2204_13254_amd.solver import DDSolver
    c, t, _ = cube_mesh(3)
    s = DDSolver(c, t, box_partition(3, 1), np.ones(len(t)), dt=0.05, beta=0.3)
    z = s.new_field()
    with pytest.raises(DDError, match="DD_ERR_STATE"):
        s.step_mixed(z, z, s.new_face_field())


def test_mixed_steps_on_slabs():
    """Slab partition (no corners, no coarse problem): the mixed step against
    the oracle in FP64."""
    from paper_2204_13254_amd.solver import DDSolver
    n = 5
    c, t, _ = cube_mesh(n)
    p = box_partition(n, (3, 1, 1))
    rng = np.random.default_rng(41)
    eps = rng.uniform(1, 3, len(t))
    mu = rng.uniform(1, 2, len(t))
    dt = 0.04
    s = DDSolver(c, t, p, eps, mu, dt=dt, beta=0.25, nrhs=2, cg_tol=1e-13, cg_max_iter=400)
    o = MixedOracle(c, t, eps=eps, mu=mu, dt=dt)
    N = 5
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, dt, 0.12, 0.04, seed=43, nrhs=2)
    b0 = np.ascontiguousarray((o.C @ rng.normal(size=(o.d.n_int, 2))).T)
    Eo, Bo = o.run(J, None, b0)
    E = torch.zeros((2, o.d.n_e), dtype=torch.float64, device="cuda")
    B = torch.tensor(b0, device="cuda")
    Jd = torch.tensor(J, device="cuda")
    for k in range(N):
        E, B = s.step_mixed(Jd[k], E, B)
        assert relerr(E.cpu().numpy(), Eo[k + 1]).max() <= 1e-10
        assert relerr(B.cpu().numpy(), Bo[k + 1]).max() <= 1e-10
