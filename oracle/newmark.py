"""Oracle, part 2: the undecomposed Newmark-beta recurrence (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Time discretisation, Sec. II-B-2: Newmark-beta with gamma = 1/2 applied to
the semi-discrete system  T e'' + S e = -j',  j_i = <W_i, J>.  Written in the
time-integrated current G = int J dt of Sec. II-A (so that j = G'), the
source's second time difference is treated exactly like the inertia term,
which gives the three-level form

    A e^{n+1} = (2A - dt^2 S) e^n - A e^{n-1} - dt (J^{n+1/2} - J^{n-1/2}),
    A = T + beta dt^2 S,

with J^{n+1/2} = (G^{n+1} - G^n)/dt the step-averaged current, e^0 = e^-1 = 0
and J^{-1/2} = 0.  Each step is solved directly: A is factorised once with
SuperLU (scipy.sparse.linalg.splu, a library primitive) and every step does
one multi-right-hand-side forward/back solve.

Also here: the discrete Gauss law G^T T e^n + q^n = 0 with
q^{n+1} = q^n + dt G^T J^{n+1/2}, the discrete energy
H^{n+1/2} = |e^{n+1}-e^n|_T^2/dt^2 + |(e^{n+1}+e^n)/2|_S^2 (constant for
beta = 1/4 without sources), and the reverse-mode adjoint of the recurrence.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .fem import Discretisation


def nested_dissection(d, leaf=2):
    """Fill-reducing order of the unknowns for the direct solve.

    Geometric nested dissection: split the edge set by the median vertex
    coordinate plane of its widest axis; edges lying in the plane form the
    separator, ordered after both halves.  Any edge that would straddle the
    plane also goes to the separator, so the result is always a permutation.
    Only the fill of the factorisation depends on this order.
    """
    e = d.edges[d.interior]
    lo = np.minimum(d.coords[e[:, 0]], d.coords[e[:, 1]])
    hi = np.maximum(d.coords[e[:, 0]], d.coords[e[:, 1]])
    out = []

    def rec(idx):                       # post-order: left, right, separator
        if len(idx) == 0:
            return
        vals = [np.unique(np.concatenate([lo[idx, a], hi[idx, a]])) for a in range(3)]
        ax = int(np.argmax([len(v) for v in vals]))
        if len(vals[ax]) <= leaf + 1:
            out.append(idx)
            return
        m = vals[ax][len(vals[ax]) // 2]
        a, b = lo[idx, ax], hi[idx, ax]
        left = (b <= m) & ~((a == m) & (b == m))
        right = (a >= m) & ~((a == m) & (b == m))
        sep = ~(left | right)
        rec(idx[left])
        rec(idx[right])
        out.append(idx[sep])
    rec(np.arange(len(e)))
    perm = np.concatenate(out)
    assert len(perm) == d.n_int and len(np.unique(perm)) == d.n_int
    return perm


def mass_lower_bound(d):
    """Certified lower bound on the smallest eigenvalue of A = T + c S (c >= 0).

    S is a sum of positive semidefinite element matrices, so x.A x >= x.T x.
    With x_k the six entries of x on the edges of tetrahedron k (zero on
    conductor edges), x.T x = sum_k eps_k x_k.T_k x_k >= sum_k eps_k
    lam_min(T_k) |x_k|^2, and every unknown lies on at least one
    tetrahedron, so sum_k |x_k|^2 >= |x|^2.  Hence
    lam_min(A) >= min_k eps_k lam_min(T_k) (T_k the unit-eps element mass).
    """
    lam = np.linalg.eigvalsh(d.unit_mass_elements())[:, 0]
    return float((d.eps * lam).min())


def pcg(A, b, x0=None, tol=1e-13, maxit=5000):
    """Conjugate gradients with the diagonal (Jacobi) preconditioner for the
    SPD matrix A and the columns of b [n, k], each column with its own
    step lengths; a column stops changing once its recursively updated
    residual is below tol ||b_col||.  The result is then re-checked with a
    freshly computed residual b - A x, and the iteration restarted from x
    while that true residual is above tol (at most 5 restarts).

    Returns (x [n, k], iterations, true relative residuals [k])."""
    A = A.tocsr()
    b = np.asarray(b, dtype=np.float64)
    dinv = 1.0 / A.diagonal()
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bn = np.linalg.norm(b, axis=0)
    bn = np.where(bn > 0, bn, 1.0)
    total = 0
    for _restart in range(6):
        r = b - A @ x
        rel = np.linalg.norm(r, axis=0) / bn
        if (rel <= tol).all():
            break
        active = rel > tol
        z = dinv[:, None] * r
        p = z.copy()
        rz = np.einsum("ij,ij->j", r, z)
        for _ in range(maxit):
            Ap = A @ p
            pAp = np.einsum("ij,ij->j", p, Ap)
            alpha = np.where(active, rz / np.where(pAp > 0, pAp, 1.0), 0.0)
            x += alpha * p
            r -= alpha * Ap
            total += 1
            active &= np.linalg.norm(r, axis=0) > tol * bn
            if not active.any():
                break
            z = dinv[:, None] * r
            rz_new = np.einsum("ij,ij->j", r, z)
            beta = np.where(active, rz_new / np.where(rz != 0, rz, 1.0), 0.0)
            p = z + beta * p
            rz = rz_new
    rel = np.linalg.norm(b - A @ x, axis=0) / bn
    return x, total, rel


class NewmarkOracle:
    """The monolithic recurrence.  solver="direct" factorises A once
    (SuperLU in a nested-dissection order); solver="pcg" solves every step
    with Jacobi-preconditioned conjugate gradients to a true relative
    residual of pcg_tol, for meshes whose factor does not fit a host, and
    records after each solve the certified error bound
    ||x - A^-1 b|| / ||x|| <= ||b - A x|| / (lam_lo ||x||), lam_lo from
    mass_lower_bound."""

    def __init__(self, coords, tets, eps=None, mu=None, dt=0.05, beta=0.25,
                 factor=True, solver="direct", pcg_tol=1e-13):
        # solver="extended": the recurrence and the assembly in 80-bit
        # extended precision (numpy longdouble), each step solved by the FP64
        # factor refined on the extended-precision residual (for finite
        # differences whose rounding floor must sit below FP64's)
        ld = solver == "extended"
        self.d = Discretisation(coords, tets, eps, mu, dtype=np.longdouble if ld else np.float64)
        self.dt = np.longdouble(dt) if ld else float(dt)
        self.beta = np.longdouble(beta) if ld else float(beta)
        d = self.d
        self.A = (d.T + (self.beta * self.dt ** 2) * d.S).tocsc()
        self.B1 = (2.0 * d.T + ((2.0 * self.beta - 1.0) * self.dt ** 2) * d.S).tocsr()
        self.lu = None
        self.solver = solver
        self.pcg_tol = float(pcg_tol)
        self.solve_log = []          # pcg: (iterations, max true relres, max error bound)
        if solver == "pcg":
            self.A = self.A.tocsr()
            self.lam_lo = mass_lower_bound(d)
        elif solver not in ("direct", "extended"):
            raise ValueError(solver)
        elif factor:
            self.perm = nested_dissection(self.d)
            Ap = self.A[self.perm][:, self.perm].astype(np.float64).tocsc()
            # A is SPD: keep the diagonal pivots, so this is a symmetric LU
            # in the given (fill-reducing) order.
            self.lu = spla.splu(Ap, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                                options=dict(SymmetricMode=True))

    # ---- one step ------------------------------------------------------------
    def rhs(self, e_n, e_nm1, J_half, J_prev_half):
        """Right-hand side on the unknowns; all arguments [nrhs, n_int]."""
        return ((self.B1 @ e_n.T).T - (self.A @ e_nm1.T).T
                - self.dt * (J_half - J_prev_half))

    def solve(self, b, x0=None):
        """A^-1 b for b [nrhs, n_int]; x0 (same shape) is the pcg start."""
        if self.solver == "pcg":
            x, it, rel = pcg(self.A, np.asarray(b).T, None if x0 is None else np.asarray(x0).T,
                             self.pcg_tol)
            xn = np.linalg.norm(x, axis=0)
            rn = rel * np.linalg.norm(np.asarray(b), axis=1)
            bound = np.where(xn > 0, rn / (self.lam_lo * np.where(xn > 0, xn, 1.0)), 0.0)
            self.solve_log.append((it, float(rel.max()), float(bound.max())))
            return np.ascontiguousarray(x.T)
        if self.solver == "extended":
            return self._solve_refined(np.asarray(b, dtype=np.longdouble))
        bp = np.ascontiguousarray(np.asarray(b).T[self.perm])
        x = np.empty_like(bp)
        x[self.perm] = self.lu.solve(bp)
        return x.T

    def _lu_solve(self, b):
        """FP64 factor applied to [nrhs, n_int] (any dtype in, float64 out)."""
        bp = np.ascontiguousarray(np.asarray(b, dtype=np.float64).T[self.perm])
        x = np.empty_like(bp)
        x[self.perm] = self.lu.solve(bp)
        return x.T

    def _solve_refined(self, b):
        """Iterative refinement to the extended-precision residual: x = LU^-1 b,
        then x += LU^-1 (b - A x) with the residual in longdouble, until it
        stops shrinking (each sweep gains the factor's ~1e-14)."""
        x = self._lu_solve(b).astype(np.longdouble)
        bn = np.linalg.norm(b.astype(np.float64), axis=1)
        prev = np.inf
        for _ in range(8):
            r = b - (self.A @ x.T).T
            rn = float(np.max(np.linalg.norm(r.astype(np.float64), axis=1) / np.where(bn > 0, bn, 1.0)))
            if rn == 0.0 or rn >= 0.5 * prev:
                break
            prev = rn
            x = x + self._lu_solve(r).astype(np.longdouble)
        self.solve_log.append((0, rn, 0.0))
        return x

    def step(self, e_n, e_nm1, J_half, J_prev_half):
        return self.solve(self.rhs(e_n, e_nm1, J_half, J_prev_half), x0=e_n)

    def run(self, J_half_edges):
        """Full history.  J_half_edges [N, nrhs, n_e] (J^{n+1/2}, n = 0..N-1).

        Returns E [N+1, nrhs, n_e] with E[0] = e^0 = 0 and E[n] = e^n.
        """
        d = self.d
        J = d.restrict(np.asarray(J_half_edges, dtype=d.dtype))
        N, nrhs, _ = J.shape
        e = np.zeros((N + 1, nrhs, d.n_int), dtype=d.dtype)
        e_nm1 = np.zeros((nrhs, d.n_int), dtype=d.dtype)
        J_prev = np.zeros((nrhs, d.n_int), dtype=d.dtype)
        for n in range(N):
            e[n + 1] = self.step(e[n], e_nm1, J[n], J_prev)
            e_nm1 = e[n]
            J_prev = J[n]
        return d.extend(e)

    def relative_residual(self, E_next, E_n, E_nm1, J_half, J_prev_half):
        """Per-RHS ||A e^{n+1} - b||_2 / ||b||_2 of the recurrence, all inputs
        as full edge arrays [nrhs, n_e].  A size-independent parity property
        for solutions computed elsewhere."""
        d = self.d
        b = self.rhs(d.restrict(E_n), d.restrict(E_nm1), d.restrict(J_half),
                     d.restrict(J_prev_half))
        r = (self.A @ d.restrict(E_next).T).T - b
        nb = np.linalg.norm(b, axis=1)
        return np.linalg.norm(r, axis=1) / np.where(nb > 0, nb, 1.0)

    # ---- diagnostics -----------------------------------------------------------
    def charge_history(self, J_half_edges):
        """q^n for n = 0..N: q^0 = 0, q^{n+1} = q^n + dt G^T J^{n+1/2}."""
        G = self.d.gradient()
        J = self.d.restrict(J_half_edges)
        N, nrhs, _ = J.shape
        q = np.zeros((N + 1, nrhs, G.shape[1]))
        for n in range(N):
            q[n + 1] = q[n] + self.dt * (G.T @ J[n].T).T
        return q

    def gauss_residual(self, E_edges, q):
        """G^T T e + q for E [nrhs, n_e], q [nrhs, n_nodes]."""
        G = self.d.gradient()
        e = self.d.restrict(E_edges)
        return (G.T @ (self.d.T @ e.T)).T + q

    def energy(self, E_next, E_n):
        """H^{n+1/2} per RHS for full edge arrays [nrhs, n_e]."""
        a = self.d.restrict(E_next)
        b = self.d.restrict(E_n)
        dv = (a - b) / self.dt
        av = 0.5 * (a + b)
        return (np.einsum("ri,ri->r", dv, (self.d.T @ dv.T).T)
                + np.einsum("ri,ri->r", av, (self.d.S @ av.T).T))

    # ---- reverse mode --------------------------------------------------------------
    def adjoint(self, J_half_edges, E_hist_edges, Ebar_final_edges):
        """Gradient of L(e^N) with respect to the currents and the per-tet
        permittivity, given dL/de^N.

        Reverse of the recurrence (A symmetric): for n = N-1 .. 0
            g^n = A^-1 ebar^{n+1};  ebar^n += B1 g^n;  ebar^{n-1} -= A g^n;
            eps_bar_k -= g^n . T_k (e^{n+1} - 2 e^n + e^{n-1})   (T_k: eps=1)
        and J^{n+1/2} enters step n with -dt and step n+1 with +dt, so
            Jbar^{n+1/2} = -dt g^n + dt g^{n+1}   (g^N = 0).
        Returns (Jbar [N, nrhs, n_e], eps_bar [n_t]).
        """
        d = self.d
        E = d.restrict(E_hist_edges)                 # [N+1, nrhs, n_int]
        N = E.shape[0] - 1
        nrhs = E.shape[1]
        ebar = np.zeros_like(E)
        ebar[N] = d.restrict(Ebar_final_edges)
        ebar_m1 = np.zeros((nrhs, d.n_int))          # adjoint of e^{-1} (unused)
        g = np.zeros((N + 1, nrhs, d.n_int))
        Tk = d.unit_mass_elements()
        dofs = d.dof[d.tet_edges]                    # [n_t, 6]
        mask = dofs >= 0
        eps_bar = np.zeros(len(d.tets))
        zero = np.zeros((nrhs, d.n_int))
        for n in range(N - 1, -1, -1):
            g[n] = self.solve(ebar[n + 1])
            ebar[n] += (self.B1 @ g[n].T).T
            if n >= 1:
                ebar[n - 1] -= (self.A @ g[n].T).T
            else:
                ebar_m1 -= (self.A @ g[n].T).T
            e_nm1 = E[n - 1] if n >= 1 else zero
            acc = E[n + 1] - 2.0 * E[n] + e_nm1       # [nrhs, n_int]
            gl = np.where(mask[None], g[n][:, np.maximum(dofs, 0)], 0.0)
            al = np.where(mask[None], acc[:, np.maximum(dofs, 0)], 0.0)
            eps_bar -= np.einsum("rta,tab,rtb->t", gl, Tk, al)
        Jbar = -self.dt * g[:N] + self.dt * g[1:N + 1]
        return d.extend(Jbar), eps_bar
