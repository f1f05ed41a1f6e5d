"""The resident Newmark state (dd_state_set, dd_step_resident): the context
keeps e^n, e^{n-1}, J^{n-1/2} and the products T e, S e of both iterates, so
a step assembles its load (Sec. II-B-2) without a sparse product.  Its
fields must equal dd_step's for the same inputs (the same kernels and sums),
and both must match the oracle: from zero, from a state loaded mid-run, after
a new permittivity (the stored products are recomputed), in FP64 and in FP32
with refinement, with the Gauss check on."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.newmark import NewmarkOracle
from workloads.mesh import cube_mesh
from workloads.partition import rcb_partition
from workloads.sources import dense_random_source

pytestmark = pytest.mark.gpu


def _case():
    c, t, _ = cube_mesh(10, 1.5)
    p = rcb_partition(10, 4, 7)
    eps = np.random.default_rng(3).uniform(1, 3, len(t))
    return c, t, p, eps


def _rel(a, b):
    return float((np.linalg.norm(a - b, axis=-1) / np.maximum(np.linalg.norm(b, axis=-1), 1e-300)).max())


@pytest.mark.parametrize("precision,nrhs,tol", [("fp32_refine", 16, 1e-8), ("fp64", 3, 1e-10)])
def test_resident_steps_equal_dd_step_and_oracle(precision, nrhs, tol):
    from paper_2204_13254_amd.solver import DDSolver
    c, t, p, eps = _case()
    dt, N = 0.03, 6
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    J = dense_random_source(o.d.n_e, ~o.d.pec, N, dt, 0.05, 0.03, seed=21, nrhs=nrhs)
    Eo = o.run(J)
    kw = dict(dt=dt, precision=precision, nrhs=nrhs, cg_tol=1e-6 if precision != "fp64" else 1e-12,
              diagnostics=1)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        a = DDSolver(c, t, p, eps, stream=st, use_graph=True, **kw)   # dd_step
        b = DDSolver(c, t, p, eps, stream=st, use_graph=True, **kw)   # resident
        Jd = torch.tensor(J, device="cuda")
        z = torch.zeros((nrhs, a.n_edges), dtype=torch.float64, device="cuda")
        Ea, Eb = [z, z.clone()], []
        for n in range(N):
            Ea.append(a.step(Jd[n], Jd[n - 1] if n else z, Ea[-1], Ea[-2], stats=True))
            sa = a.last_stats()
            Eb.append(b.step_resident(Jd[n], stats=True))
            sb = b.last_stats()
            # the same accumulated charge; residuals at rounding level on both
            assert sa["charge_max"] == sb["charge_max"], n
            q = np.array(sb["charge_max"])
            assert np.all(np.array(sb["gauss_residual"]) <= 1e-9 * q), (n, sb["gauss_residual"], q)
        st.synchronize()
    A = torch.stack(Ea[2:]).cpu().numpy()
    B = torch.stack(Eb).cpu().numpy()
    d = float(np.abs(A - B).max())
    print(f"{precision}: max |resident - dd_step| = {d:.3e}", flush=True)
    # the same kernels sum the same products in the same order; a bound at the
    # refinement tolerance leaves room for a contraction the compiler may
    # place differently in the load kernel
    assert d <= 1e-12 * np.abs(A).max()
    assert max(_rel(B[k], Eo[k + 1]) for k in range(N)) <= tol


def test_resident_state_set_and_new_eps():
    """State loaded from fields produced by dd_step (mid-run), then steps on
    both paths; then a new permittivity on both contexts (new factors, the
    resident products recomputed) and more steps, each against dd_step."""
    from paper_2204_13254_amd.solver import DDSolver
    c, t, p, eps = _case()
    dt, nrhs = 0.03, 16
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    J = dense_random_source(o.d.n_e, ~o.d.pec, 8, dt, 0.05, 0.03, seed=23, nrhs=nrhs)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        kw = dict(dt=dt, precision="fp32_refine", nrhs=nrhs, cg_tol=1e-6, stream=st, use_graph=True)
        a = DDSolver(c, t, p, eps, **kw)
        b = DDSolver(c, t, p, eps, **kw)
        Jd = torch.tensor(J, device="cuda")
        z = torch.zeros((nrhs, a.n_edges), dtype=torch.float64, device="cuda")
        E = [z, z.clone()]
        for n in range(3):
            E.append(a.step(Jd[n], Jd[n - 1] if n else z, E[-1], E[-2]))
        b.state_set(E[-1], E[-2], Jd[2])
        for n in range(3, 5):
            E.append(a.step(Jd[n], Jd[n - 1], E[-1], E[-2]))
            Eb = b.step_resident(Jd[n])
            assert float((Eb - E[-1]).abs().max()) <= 1e-12 * float(E[-1].abs().max()), n
        eps2 = eps * np.random.default_rng(4).uniform(0.9, 1.1, len(eps))
        for x in (a, b):
            x.set_eps(eps2)
            x.factor()
        for n in range(5, 8):
            E.append(a.step(Jd[n], Jd[n - 1], E[-1], E[-2]))
            Eb = b.step_resident(Jd[n])
            assert float((Eb - E[-1]).abs().max()) <= 1e-12 * float(E[-1].abs().max()), n
        st.synchronize()
