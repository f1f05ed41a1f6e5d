"""Oracle, part 4: the mixed E/B system on edges and faces (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain and monolithic:
the whole block system is factorised once with SuperLU (a library
primitive) and every step is one solve.

Sec. II-B-1 discretises E in Whitney 1-forms (edges) and B in Whitney
2-forms (faces).  For a face with vertices i < j < k (normal by the
right-hand rule i -> j -> k) the 2-form basis function is

    W_ijk = 2 (lam_i g_j x g_k + lam_j g_k x g_i + lam_k g_i x g_j),

and the discrete curl C (faces x edges) maps the boundary of face (i, j, k)
to (i,j) + (j,k) - (i,k).  Faraday's law holds exactly in these spaces,
db/dt = -C e, and Ampere's law tested with the edge functions reads
T de/dt = C^T M b - j, with M the 1/mu-weighted 2-form mass matrix (so
C^T M C is the curl-curl matrix S of the edge-only form).

Time discretisation: the trapezoid rule on both laws (the gamma = 1/2,
beta = 1/4 member of the Newmark family of Sec. II-B-2; the coefficients the
paper prints for its mixed form are not consistent with each other):

    T (e+ - e)/dt = C^T M (b+ + b)/2 - J^{n+1/2},
    (b+ - b)/dt   = -C (e+ + e)/2,

with J^{n+1/2} the step-averaged edge current.  Outer boundary: perfect
conductor; edges on it carry no unknown, faces keep their (zero) flux.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Discretisation, barycentric_gradients, sort_tets

# faces of a tetrahedron with sorted vertices: the face opposite local vertex
# k, its vertices ascending
LOCAL_FACES = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))


def canonical_faces(tets):
    """Faces (a < b < c) numbered lexicographically, and tet_faces [n_t, 4]:
    the face opposite local vertex k of each sorted tetrahedron."""
    st = sort_tets(tets)
    nv = int(st.max()) + 1
    keys = np.stack([(st[:, a] * nv + st[:, b]) * nv + st[:, c] for a, b, c in LOCAL_FACES], axis=1)
    uniq, inv = np.unique(keys.ravel(), return_inverse=True)
    faces = np.stack([uniq // (nv * nv), (uniq // nv) % nv, uniq % nv], axis=1)
    return faces, inv.reshape(-1, 4)


def curl_incidence(edges, faces):
    """C [n_f, n_e]: +1 on edges (a,b) and (b,c), -1 on (a,c) of face (a,b,c)."""
    edges = np.asarray(edges, dtype=np.int64)
    faces = np.asarray(faces, dtype=np.int64)
    nv = int(max(edges.max(), faces.max())) + 1
    ekey = edges[:, 0] * nv + edges[:, 1]                  # ascending (canonical order)
    a, b, c = faces[:, 0], faces[:, 1], faces[:, 2]
    cols = [np.searchsorted(ekey, p * nv + q) for p, q in ((a, b), (b, c), (a, c))]
    for k, (p, q) in zip(cols, ((a, b), (b, c), (a, c))):
        assert np.array_equal(ekey[k], p * nv + q)
    nf = len(faces)
    rows = np.tile(np.arange(nf), 3)
    vals = np.concatenate([np.ones(nf), np.ones(nf), -np.ones(nf)])
    return sp.csr_matrix((vals, (rows, np.concatenate(cols))), shape=(nf, len(edges)))


def face_mass_elements(coords, tets, mu=None):
    """Per-tet 2-form mass [n_t, 4, 4] over LOCAL_FACES:
    int mu^-1 W_f . W_g, with int lam_a lam_b = V (1 + delta_ab) / 20."""
    g, vol = barycentric_gradients(coords, tets)
    nt = len(vol)
    mu = np.ones(nt) if mu is None else np.asarray(mu, dtype=np.float64)

    def coeffs(face):
        i, j, k = face
        return {i: np.cross(g[:, j], g[:, k]), j: np.cross(g[:, k], g[:, i]), k: np.cross(g[:, i], g[:, j])}

    cf = [coeffs(f) for f in LOCAL_FACES]
    M = np.zeros((nt, 4, 4))
    for F in range(4):
        for G in range(4):
            s = np.zeros(nt)
            for a, ca in cf[F].items():
                for b, cb in cf[G].items():
                    s += (2.0 if a == b else 1.0) / 20.0 * np.einsum("td,td->t", ca, cb)
            M[:, F, G] = 4.0 * vol * s
    return M / mu[:, None, None]


class MixedOracle:
    """Monolithic trapezoid step of the mixed system; e on the interior
    edges (PEC edges zero), b on all faces."""

    def __init__(self, coords, tets, eps=None, mu=None, dt=0.05, factor=True):
        self.d = Discretisation(coords, tets, eps, mu)
        d = self.d
        self.dt = float(dt)
        self.faces, self.tet_faces = canonical_faces(tets)
        self.n_f = len(self.faces)
        Cfull = curl_incidence(d.edges, self.faces)
        self.C = Cfull[:, d.interior].tocsr()                      # faces x unknowns
        Me = face_mass_elements(coords, tets, mu)
        tf = self.tet_faces
        rows = np.repeat(tf, 4, axis=1).ravel()
        cols = np.tile(tf, (1, 4)).ravel()
        self.M = sp.coo_matrix((Me.reshape(-1), (rows, cols)), shape=(self.n_f, self.n_f)).tocsr()
        self.M.sum_duplicates()
        dt = self.dt
        CtM = (self.C.T @ self.M).tocsr()
        self.CtM = CtM
        self.lu = None
        if factor:
            K = sp.bmat([[d.T / dt, -0.5 * CtM], [0.5 * self.C, sp.identity(self.n_f) / dt]], format="csc")
            self.lu = spla.splu(K)

    def step(self, e, b, J):
        """One step for e [nrhs, n_int], b [nrhs, n_f], J [nrhs, n_int]."""
        dt = self.dt
        r1 = (self.d.T @ e.T).T / dt + 0.5 * (self.CtM @ b.T).T - J
        r2 = b / dt - 0.5 * (self.C @ e.T).T
        x = self.lu.solve(np.ascontiguousarray(np.concatenate([r1, r2], axis=1).T))
        x = x.T
        n = self.d.n_int
        return x[:, :n], x[:, n:]

    def run(self, J_half_edges, e0=None, b0=None):
        """J [N, nrhs, n_e] -> E [N+1, nrhs, n_e], B [N+1, nrhs, n_f]."""
        d = self.d
        J = d.restrict(J_half_edges)
        N, nrhs, _ = J.shape
        e = np.zeros((nrhs, d.n_int)) if e0 is None else d.restrict(e0)
        b = np.zeros((nrhs, self.n_f)) if b0 is None else np.asarray(b0, dtype=np.float64)
        Es, Bs = [d.extend(e)], [b.copy()]
        for n in range(N):
            e, b = self.step(e, b, J[n])
            Es.append(d.extend(e))
            Bs.append(b.copy())
        return np.stack(Es), np.stack(Bs)

    # ---- properties for solutions computed elsewhere (any size) -----------------
    def eliminated_residual(self, E_next, E_n, B_n, J_half):
        """Per-RHS ||A e+ - r|| / ||r|| of the edge equation left after
        eliminating b+, A = T + dt^2/4 S, r = (T - dt^2/4 S) e + dt C^T M b - dt J
        (full edge arrays for E and J, face arrays for B)."""
        d, dt = self.d, self.dt
        e1, e0, J = d.restrict(E_next), d.restrict(E_n), d.restrict(J_half)
        q = 0.25 * dt * dt
        r = (d.T @ e0.T).T - q * (d.S @ e0.T).T + dt * (self.CtM @ np.asarray(B_n).T).T - dt * J
        res = (d.T @ e1.T).T + q * (d.S @ e1.T).T - r
        nr = np.linalg.norm(r, axis=1)
        return np.linalg.norm(res, axis=1) / np.where(nr > 0, nr, 1.0)

    def face_update_residual(self, E_next, E_n, B_n, B_next):
        """max |b+ - b + dt/2 C (e+ + e)| per RHS."""
        d = self.d
        s = d.restrict(E_next) + d.restrict(E_n)
        res = np.asarray(B_next) - np.asarray(B_n) + 0.5 * self.dt * (self.C @ s.T).T
        return np.abs(res).max(axis=1)

    def energy(self, E_edges, B):
        """(e^T T e + b^T M b) / 2 per RHS."""
        e = self.d.restrict(E_edges)
        return 0.5 * (np.einsum("ri,ri->r", e, (self.d.T @ e.T).T) + np.einsum("ri,ri->r", B, (self.M @ B.T).T))
