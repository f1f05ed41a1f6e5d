"""GPU parity of the particle steps (dd_pic_* through the C ABI) against the
FP64 oracle (oracle/pic.py): point location, the exact current mapping of
Sec. II-A, Faraday's per-tetrahedron update, Whitney interpolation with the
Adams-Bashforth push, and a short closed PIC cycle through the decomposed
field solve with the discrete Gauss law checked at every step.  At the
64^3 beam size the deposit is checked against the structured Kuhn-plane
deposit of the source generator (a different algorithm), against the oracle
on sampled single paths, and through the discrete continuity equation.

Tolerances: deposit and fields 1e-12 relative to the largest entry (FP64 on
both sides; the GPU sums particles in an unfixed order); closed cycle 1e-10
(the field solve's CG tolerance 1e-12 enters every step)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import pic
from oracle.newmark import NewmarkOracle
from workloads.beam import BeamSampler, deposit as kuhn_deposit
from workloads.mesh import centred_cube_mesh, cube_mesh, jittered_cube_mesh, mesh_edges
from workloads.partition import box_partition
from workloads.sources import dense_random_source

pytestmark = pytest.mark.gpu


def _solver(c, t, parts, dt=0.05, factor=False, **k):
    from paper_2204_13254_amd.solver import DDSolver
    n = round(len(t) ** (1 / 3) / 6 ** (1 / 3))
    p = box_partition(n, parts)
    return DDSolver(c, t, p, np.ones(len(t)), dt=dt, factor=factor, **k)


def _locate(s, x, cell=None):
    c = s.pic_locate(x, cell)
    return c, s.pic_status()["absorbed_or_outside"]


def _deposit(s, *args):
    """Deposit, then the number of absorbed particles (no other counter set)."""
    s.pic_deposit(*args)
    st = s.pic_status()
    assert st["walk_cap"] == 0 and st["bad_index"] == 0, st
    return st["absorbed_or_outside"]


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def jm5():
    c, t, _ = jittered_cube_mesh(5, 0.2, 11)
    return c, t, pic.TetMesh(c, t)


def _wall_exit(a, b):
    """Parameter where a -> b leaves the unit cube (1 if it stays inside)."""
    d = b - a
    s = np.ones(len(a))
    for ax in range(3):
        with np.errstate(divide="ignore", invalid="ignore"):
            hi = np.where(d[:, ax] > 0, (1.0 - a[:, ax]) / d[:, ax], np.inf)
            lo = np.where(d[:, ax] < 0, -a[:, ax] / d[:, ax], np.inf)
        s = np.minimum(s, np.minimum(hi, lo))
    return s


def test_locate(jm5):
    c, t, mesh = jm5
    s = _solver(c, t, 2)
    rng = np.random.default_rng(0)
    X = np.concatenate([rng.uniform(0.0, 1.0, (3000, 3)), [[1.5, 0.5, 0.5], [0.5, -0.1, 0.5]]])
    cell, nout = _locate(s, _dev(X))
    cell = _host(cell)
    assert nout == 2 and (cell[-2:] == -1).all()
    ref = pic.locate(mesh, X[:-2])
    assert (cell[:-2] >= 0).all()
    # the located tetrahedron holds the point; where the point is clearly
    # inside one tetrahedron (not near a face) the index is unique
    lam = np.array([mesh.lam(x, np.array([k]))[0] for x, k in zip(X[:-2], cell[:-2])])
    assert lam.min() >= -1e-12
    deep = lam.min(axis=1) > 1e-9
    assert np.array_equal(cell[:-2][deep], ref[deep])
    # start from a given cell, and the empty call
    cell2, _ = _locate(s, _dev(X[:-2]), _dev(ref[::-1].copy(), torch.int32))
    assert np.array_equal(_host(cell2)[deep], ref[deep])
    e, n0 = _locate(s, _dev(np.zeros((0, 3))))
    assert n0 == 0 and e.numel() == 0


def test_deposit_parity(jm5):
    c, t, mesh = jm5
    dt = 0.05
    s = _solver(c, t, 2, dt=dt)
    rng = np.random.default_rng(1)
    m = 400
    A = rng.uniform(0.02, 0.98, (m, 3))
    L = np.concatenate([rng.uniform(0.0, 0.05, m // 2), rng.uniform(0.05, 0.6, m - m // 2)])
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    B = A + d * L[:, None]
    B[-10:] = A[-10:]                      # zero-length paths
    q = rng.uniform(-1, 1, m)
    sw = _wall_exit(A, B)                  # paths that hit the wall are cut there
    out = sw < 1.0
    Bc = np.where(out[:, None], A + (B - A) * sw[:, None], B)
    cell, _ = _locate(s, _dev(A))
    cell_h = _host(cell).copy()
    cell_h[5] = -1                         # inactive particle: skipped
    keep = np.ones(m, bool)
    keep[5] = False
    cell = _dev(cell_h, torch.int32)
    J = torch.zeros(s.n_edges, dtype=torch.float64, device="cuda")
    nabs = _deposit(s, _dev(A), _dev(B), _dev(q), cell, J)
    Jg = _host(J)
    Jo = pic.deposit(mesh, A[keep], Bc[keep], q[keep], dt)
    scale = np.abs(Jo).max()
    assert out.sum() > 20
    np.testing.assert_allclose(Jg, Jo, rtol=0, atol=1e-12 * scale)
    assert nabs == int((out & keep).sum())
    ce = _host(cell)
    assert (ce[out & keep] == -1).all() and ce[5] == -1
    inside = ~out & keep
    lam = np.array([mesh.lam(x, np.array([k]))[0] for x, k in zip(B[inside], ce[inside])])
    assert lam.min() >= -1e-12
    # empty call leaves J alone
    s.pic_deposit(_dev(np.zeros((0, 3))), _dev(np.zeros((0, 3))), _dev(np.zeros(0)),
                  _dev(np.zeros(0), torch.int32), J)
    np.testing.assert_array_equal(_host(J), Jg)


def test_sort_and_permute(jm5):
    c, t, mesh = jm5
    s = _solver(c, t, 2)
    rng = np.random.default_rng(7)
    n = 20000
    cells = rng.integers(-1, len(t), n).astype(np.int32)
    cells[:50] = len(t) + 5                 # out of range: ordered with the inactive ones
    cd = _dev(cells, torch.int32)
    perm = _host(s.pic_sort(cd))
    assert np.array_equal(np.sort(perm), np.arange(n))
    key = np.where((cells < 0) | (cells >= len(t)), len(t), cells)
    assert (np.diff(key[perm]) >= 0).all()
    P = _dev(perm, torch.int32)
    X = rng.normal(size=(n, 3))
    H = rng.normal(size=(n, 6))
    np.testing.assert_array_equal(_host(s.pic_permute(P, _dev(X))), X[perm])
    np.testing.assert_array_equal(_host(s.pic_permute(P, _dev(H))), H[perm])
    np.testing.assert_array_equal(_host(s.pic_permute(P, cd)), cells[perm])
    assert _host(s.pic_sort(_dev(np.zeros(0), torch.int32))).size == 0


@pytest.mark.parametrize("order", ["random", "by_cell"])
def test_deposit_many_per_cell(jm5, order):
    """Thousands of short paths on 750 tetrahedra (about 4 per start cell):
    in random order duplicate cells sit in non-adjacent lanes, in cell order
    they form runs that the wavefront sums before its atomics."""
    c, t, mesh = jm5
    dt = 0.02
    s = _solver(c, t, 2, dt=dt)
    rng = np.random.default_rng(8)
    m = 3000
    A = rng.uniform(0.01, 0.99, (m, 3))
    B = np.clip(A + rng.normal(0, 0.03, (m, 3)), 0.001, 0.999)
    q = rng.uniform(-1, 1, m)
    cell, _ = _locate(s, _dev(A))
    a, b, qd = _dev(A), _dev(B), _dev(q)
    if order == "by_cell":
        perm = s.pic_sort(cell)
        a, b, qd, cell = (s.pic_permute(perm, z) for z in (a, b, qd, cell))
        ch = _host(cell)
        assert (np.diff(ch) >= 0).all() and (np.diff(ch) == 0).mean() > 0.5
    J = torch.zeros(s.n_edges, dtype=torch.float64, device="cuda")
    assert _deposit(s, a, b, qd, cell, J) == 0
    Jo = pic.deposit(mesh, A, B, q, dt)
    np.testing.assert_allclose(_host(J), Jo, rtol=0, atol=1e-12 * np.abs(Jo).max())


def test_bad_indices_are_counted(jm5):
    c, t, mesh = jm5
    s = _solver(c, t, 2)
    x = _dev(np.full((2, 3), 0.5))
    cell = _dev(np.array([0, len(t) + 3]), torch.int32)
    J = torch.zeros(s.n_edges, dtype=torch.float64, device="cuda")
    s.pic_deposit(x, x, _dev(np.ones(2)), cell, J)
    st = s.pic_status()
    assert st == {"absorbed_or_outside": 0, "walk_cap": 0, "bad_index": 1}
    assert _host(cell)[1] == -1 and s.pic_status()["bad_index"] == 0   # reset
    perm = _dev(np.array([1, 7]), torch.int32)
    out = torch.full((2,), -5.0, dtype=torch.float64, device="cuda")
    s.pic_permute(perm, _dev(np.array([3.0, 4.0])), out)
    assert s.pic_status()["bad_index"] == 1
    np.testing.assert_array_equal(_host(out), [4.0, -5.0])


def test_faraday_parity(jm5):
    c, t, mesh = jm5
    s = _solver(c, t, 2)
    rng = np.random.default_rng(2)
    e = rng.normal(size=s.n_edges)
    B0 = rng.normal(size=(len(t), 3))
    B = _dev(B0)
    s.pic_faraday(_dev(e), -0.37, B)
    ref = pic.faraday(mesh, e, B0, -0.37)
    np.testing.assert_allclose(_host(B), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # three right-hand sides in one call
    e3 = rng.normal(size=(3, s.n_edges))
    B3 = rng.normal(size=(3, len(t), 3))
    Bd = _dev(B3)
    s.pic_faraday(_dev(e3), 0.25, Bd)
    for r in range(3):
        ref = pic.faraday(mesh, e3[r], B3[r], 0.25)
        np.testing.assert_allclose(_host(Bd)[r], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_push_parity(jm5):
    c, t, mesh = jm5
    dt = 0.04
    s = _solver(c, t, 2, dt=dt)
    rng = np.random.default_rng(3)
    m = 1000
    X = rng.uniform(0.05, 0.95, (m, 3))
    V = rng.normal(0, 0.5, (m, 3))
    qm = rng.uniform(-3, 3, m)
    e = rng.normal(size=s.n_edges)
    Bt = rng.normal(size=(len(t), 3))
    cell, _ = _locate(s, _dev(X))
    ch = _host(cell).copy()
    ch[7] = -1
    cell = _dev(ch, torch.int32)
    x, v, hist = _dev(X), _dev(V), torch.zeros((m, 6), dtype=torch.float64, device="cuda")
    xn = torch.empty_like(x)
    act = ch >= 0
    # oracle, two steps from the same cells (the push does not move cells)
    xo, vo, hv, ha = X[act].copy(), V[act].copy(), None, None
    for first in (True, False):
        s.pic_push(_dev(qm), _dev(e), _dev(Bt), cell, x, xn, v, hist, first)
        E = pic.whitney_field(mesh, e, ch[act], xo)
        acc = pic.lorentz(qm[act], E, Bt[ch[act]], vo)
        xo, vo, hv, ha = pic.push_ab2(xo, vo, acc, hv, ha, dt, first)
        xg, vg, hg = _host(xn), _host(v), _host(hist)
        np.testing.assert_allclose(xg[act], xo, rtol=0, atol=1e-13)
        np.testing.assert_allclose(vg[act], vo, rtol=0, atol=1e-12 * np.abs(vo).max())
        np.testing.assert_allclose(hg[act, 3:], ha, rtol=0, atol=1e-12 * np.abs(ha).max())
        np.testing.assert_allclose(hg[act, :3], hv, rtol=0, atol=1e-13 * np.abs(hv).max())
        assert np.array_equal(xg[7], X[7]) and np.array_equal(vg[7], V[7])
        x = xn.clone()


def test_closed_cycle_with_gauss_law():
    """push (E^n, B^n) -> deposit x^n -> x^{n+1} -> field step -> Faraday
    (trapezoid in E) on a jittered 6^3 mesh with 8 subdomains, plus a dense
    external current so that E is not small; GPU vs oracle at every step, and
    the interior Gauss law G^T T e^n + q^n = 0 on the GPU."""
    n, dt, steps, m = 6, 0.05, 6, 150
    c, t, _ = jittered_cube_mesh(n, 0.15, 21)
    mesh = pic.TetMesh(c, t)
    s = _solver(c, t, 2, dt=dt, factor=True, cg_tol=1e-12)
    o = NewmarkOracle(c, t, dt=dt)
    rng = np.random.default_rng(4)
    X0 = rng.uniform(0.3, 0.7, (m, 3))
    V0 = rng.normal(0, 0.3, (m, 3))
    q = rng.choice([-1.0, 1.0], m) * 0.02
    qm = np.sign(q) * 4.0
    Bt0 = np.tile([0.0, 0.0, 1.5], (len(t), 1))
    edges = mesh_edges(t)
    from workloads.mesh import boundary_edge_mask
    Jx = 0.05 * dense_random_source(len(edges), ~boundary_edge_mask(c, edges), steps, dt, 0.1, 0.05, 9)[:, 0]

    # ---- GPU -------------------------------------------------------------------
    x, v = _dev(X0), _dev(V0)
    hist = torch.zeros((m, 6), dtype=torch.float64, device="cuda")
    xn = torch.empty_like(x)
    cell, nout = _locate(s, x)
    assert nout == 0
    Bg = _dev(Bt0)
    e_n = s.new_field(); e_nm1 = s.new_field(); J_prev = s.new_field()
    qn = torch.zeros((1, len(c)), dtype=torch.float64, device="cuda")
    # ---- oracle ----------------------------------------------------------------
    xo, vo, hv, ha = X0.copy(), V0.copy(), None, None
    Bo = Bt0.copy()
    eo = np.zeros((1, o.d.n_e)); eo_m1 = np.zeros_like(eo); Jo_prev = np.zeros_like(eo)
    for k in range(steps):
        s.pic_push(_dev(qm), e_n[0], Bg, cell, x, xn, v, hist, k == 0)
        J = _dev(Jx[k][None, :])
        s.pic_deposit(x, xn, _dev(q), cell, J[0])
        e_next = s.step(J, J_prev, e_n, e_nm1)
        s.pic_faraday(e_n[0], -0.5 * dt, Bg)
        s.pic_faraday(e_next[0], -0.5 * dt, Bg)
        s.charge_update(J, qn)
        res = s.gauss_residual(e_next, qn)
        x, xn = xn, x
        e_nm1, e_n, J_prev = e_n, e_next, J

        cells_o = pic.locate(mesh, xo)
        E = pic.whitney_field(mesh, eo[0], cells_o, xo)
        acc = pic.lorentz(qm, E, Bo[cells_o], vo)
        xo1, vo, hv, ha = pic.push_ab2(xo, vo, acc, hv, ha, dt, k == 0)
        Jo = Jx[k][None, :] + pic.deposit(mesh, xo, xo1, q, dt)[None, :]
        d = o.d
        en = d.extend(o.step(d.restrict(eo), d.restrict(eo_m1), d.restrict(Jo), d.restrict(Jo_prev)))
        Bo = pic.faraday(mesh, eo[0], Bo, -0.5 * dt)
        Bo = pic.faraday(mesh, en[0], Bo, -0.5 * dt)
        xo, eo_m1, eo, Jo_prev = xo1, eo, en, Jo

        tol = 1e-10
        np.testing.assert_allclose(_host(x), xo, rtol=0, atol=tol)
        np.testing.assert_allclose(_host(v), vo, rtol=0, atol=tol * np.abs(vo).max())
        eg = _host(e_n)
        assert np.linalg.norm(eg - eo) <= tol * np.linalg.norm(eo)
        np.testing.assert_allclose(_host(Bg), Bo, rtol=0, atol=tol * np.abs(Bo).max())
        qs = np.abs(_host(qn)).max()
        assert res[0] <= 1e-10 * max(qs, 1e-30), (k, res, qs)
    assert np.abs(eo).max() > 0 and np.abs(_host(v) - V0).max() > 1e-3


def test_beam_fullsize_deposit():
    """One right-hand side of the 64^3 beam workload (1e6 particles, dt
    0.008): GPU deposit vs the structured Kuhn-plane deposit, the sampled
    single-path oracle, and the discrete continuity equation."""
    n, dt = 64, 0.008
    c, t, _ = cube_mesh(n)
    s = _solver(c, t, (10, 10, 10), dt=dt)
    bs = BeamSampler(n, 1_000_000, 0.2, 0.01, 0.3, 1e-6, 1000)
    step = 37
    a = bs.x0 + bs.v * (step * dt)
    b = bs.x0 + bs.v * ((step + 1) * dt)
    wrap = np.floor(b[:, 2]) > np.floor(a[:, 2])   # re-entry at z = 0: not this path
    a, b = a[~wrap], b[~wrap]
    w = np.floor(a[:, 2])
    a[:, 2] -= w
    b[:, 2] -= w
    q = bs.q[~wrap]
    print(f"beam paths {len(a)}", flush=True)
    cell, nout = _locate(s, _dev(a))
    assert nout == 0
    cell0 = _host(cell).copy()
    J = torch.zeros(s.n_edges, dtype=torch.float64, device="cuda")
    nabs = _deposit(s, _dev(a), _dev(b), _dev(q), cell, J)
    assert nabs == 0
    Jg = _host(J)
    edges, _ = s.edges()
    nv1 = len(c)
    keys = edges[:, 0].astype(np.int64) * nv1 + edges[:, 1]
    K = kuhn_deposit(n, keys, nv1, a, b, q, dt, len(edges))
    scale = np.abs(K).max()
    np.testing.assert_allclose(Jg, K, rtol=0, atol=1e-12 * scale)
    # the same paths in cell order (long runs of equal start cells)
    perm = s.pic_sort(_dev(cell0, torch.int32))
    ad, bd, qd, cd = (s.pic_permute(perm, z) for z in (_dev(a), _dev(b), _dev(q), _dev(cell0, torch.int32)))
    J2 = torch.zeros(s.n_edges, dtype=torch.float64, device="cuda")
    assert _deposit(s, ad, bd, qd, cd, J2) == 0
    np.testing.assert_allclose(_host(J2), K, rtol=0, atol=1e-12 * scale)
    # continuity: dt G^T J = sum_p q_p (lam(b) - lam(a)) at every vertex
    mesh = pic.TetMesh(c, t)
    ce = _host(cell)

    def hats(x, cl):
        L = np.einsum("pkd,pd->pk", mesh.g[cl], x - mesh.x0[cl])
        L[:, 0] += 1.0
        return mesh.st[cl], L

    vb, wb = hats(b, ce)
    va, wa = hats(a, cell0)
    assert wb.min() >= -1e-12 and wa.min() >= -1e-12
    ref = np.zeros(nv1)
    np.add.at(ref, vb.ravel(), (q[:, None] * wb).ravel())
    np.add.at(ref, va.ravel(), -(q[:, None] * wa).ravel())
    div = np.zeros(nv1)
    np.add.at(div, edges[:, 1], Jg * dt)
    np.add.at(div, edges[:, 0], -Jg * dt)
    np.testing.assert_allclose(div, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # sampled single paths against the oracle
    rng = np.random.default_rng(6)
    for p in rng.choice(len(a), 6, replace=False):
        J1 = torch.zeros(s.n_edges, dtype=torch.float64, device="cuda")
        c1 = _dev(cell0[p:p + 1], torch.int32)
        s.pic_deposit(_dev(a[p:p + 1]), _dev(b[p:p + 1]), _dev(q[p:p + 1]), c1, J1)
        Jo = pic.deposit(mesh, a[p], b[p], q[p], dt)
        np.testing.assert_allclose(_host(J1), Jo, rtol=0, atol=1e-12 * np.abs(Jo).max())


def test_locate_and_deposit_on_centred_mesh():
    """Another topology: cubes cut into 12 tetrahedra around their centres
    (vertices shared by up to 24 tetrahedra, centre vertices by 12).  Location
    and the exact deposit of long paths (crossing many cells, through the
    added centres' neighbourhoods) against the brute-force oracle."""
    from paper_2204_13254_amd.solver import DDSolver
    n = 4
    c, t, _ = centred_cube_mesh(n)
    mesh = pic.TetMesh(c, t)
    p = np.repeat(box_partition(n, 2)[::6], 12)
    dt = 0.05
    s = DDSolver(c, t, p, np.ones(len(t)), dt=dt, factor=False)
    rng = np.random.default_rng(31)
    m = 300
    A = rng.uniform(0.03, 0.97, (m, 3))
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    B = A + d * rng.uniform(0.0, 0.5, m)[:, None]
    sw = _wall_exit(A, B)
    out = sw < 1.0
    Bc = np.where(out[:, None], A + (B - A) * sw[:, None], B)
    q = rng.uniform(-1, 1, m)
    cell, nout = _locate(s, _dev(A))
    ch = _host(cell)
    assert nout == 0
    lam = np.array([mesh.lam(x, np.array([k]))[0] for x, k in zip(A, ch)])
    assert lam.min() >= -1e-12
    J = torch.zeros(s.n_edges, dtype=torch.float64, device="cuda")
    nabs = _deposit(s, _dev(A), _dev(B), _dev(q), cell, J)
    Jo = pic.deposit(mesh, A, Bc, q, dt)
    np.testing.assert_allclose(_host(J), Jo, rtol=0, atol=1e-12 * np.abs(Jo).max())
    assert nabs == int(out.sum()) and out.sum() > 10
