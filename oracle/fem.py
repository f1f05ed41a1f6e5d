"""Oracle, part 1: edges, Whitney element matrices, global assembly (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain, slow on purpose.

Spatial discretisation, Sec. II-B-1: the electric field is expanded in
Whitney 1-forms W_ij = lam_i grad(lam_j) - lam_j grad(lam_i), one per edge
(i, j) of a tetrahedron, with lam the barycentric coordinates.  Testing the
edge-only wave equation eps d2E/dt2 + curl(mu^-1 curl E) = -dJ/dt with the
same functions gives the mass matrix T (entries <eps W_a, W_b>) and the
curl-curl matrix S (entries <mu^-1 curl W_a, curl W_b>).  Only the B unknowns
of the paper's mixed system are eliminated (Sec. V names this edge-only form
as the way to shrink the unknown count); outer boundary: perfect conductor,
so edges on the boundary carry no unknown.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# Local edges of a tetrahedron whose vertices are sorted ascending, each
# oriented from the lower to the higher global vertex id.
LOCAL_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def sort_tets(tets):
    """Vertices of each tetrahedron in ascending global id."""
    return np.sort(np.asarray(tets, dtype=np.int64), axis=1)


def canonical_edges(tets):
    """Edges (v_lo, v_hi), v_lo < v_hi, numbered lexicographically.

    Returns (edges [n_e, 2] int64, tet_edges [n_t, 6] int64): tet_edges[t, a]
    is the global id of local edge LOCAL_EDGES[a] of sorted tetrahedron t.
    Because the vertices are sorted, local and global orientations agree.
    """
    st = sort_tets(tets)
    nv = int(st.max()) + 1
    keys = np.stack([st[:, a] * nv + st[:, b] for a, b in LOCAL_EDGES], axis=1)
    uniq, inv = np.unique(keys.ravel(), return_inverse=True)
    edges = np.stack([uniq // nv, uniq % nv], axis=1)
    return edges, inv.reshape(-1, 6)


def pec_mask(coords, edges):
    """An edge is on the perfect conductor iff both end points lie on the
    same face of the unit cube (same axis, coordinate exactly 0 or 1)."""
    a = coords[edges[:, 0]]
    b = coords[edges[:, 1]]
    m = np.zeros(len(edges), dtype=bool)
    for ax in range(3):
        for v in (0.0, 1.0):
            m |= (a[:, ax] == v) & (b[:, ax] == v)
    return m


def _inv3(D):
    """Inverse and determinant of 3x3 matrices [n, 3, 3] by cofactors (any
    float dtype: LAPACK has no extended precision)."""
    a = D
    cof = np.empty_like(a)
    for i in range(3):
        for j in range(3):
            r = [k for k in range(3) if k != i]
            c = [k for k in range(3) if k != j]
            m = a[:, r[0], c[0]] * a[:, r[1], c[1]] - a[:, r[0], c[1]] * a[:, r[1], c[0]]
            cof[:, i, j] = m if (i + j) % 2 == 0 else -m
    det = np.einsum("nj,nj->n", a[:, 0, :], cof[:, 0, :])
    return cof.transpose(0, 2, 1) / det[:, None, None], det


def barycentric_gradients(coords, tets):
    """Gradients g[t, i] of lam_i (constant per tetrahedron) and volumes, in
    the dtype of coords (float64 through LAPACK, others by cofactors)."""
    st = sort_tets(tets)
    x = coords[st]                      # [n_t, 4, 3]
    D = (x[:, 1:, :] - x[:, :1, :]).transpose(0, 2, 1)   # columns x_i - x_0
    if D.dtype == np.float64:
        det = np.linalg.det(D)
        Dinv = np.linalg.inv(D)         # rows = grad lam_1..3
    else:
        Dinv, det = _inv3(D)
    g = np.empty((len(st), 4, 3), dtype=D.dtype)
    g[:, 1:, :] = Dinv
    g[:, 0, :] = -Dinv.sum(axis=1)
    vol = np.abs(det) / 6.0
    return g, vol


def element_matrices(coords, tets, eps=None, mu=None):
    """Whitney element mass T_e and curl-curl S_e, shape [n_t, 6, 6].

    T_e[(ij),(kl)] = eps * integral (lam_i g_j - lam_j g_i).(lam_k g_l - lam_l g_k)
      with integral lam_a lam_b dV = V (1 + delta_ab) / 20;
    S_e[(ij),(kl)] = mu^-1 * integral (2 g_i x g_j).(2 g_k x g_l) dV.
    """
    g, vol = barycentric_gradients(coords, tets)
    nt = len(vol)
    dt_ = vol.dtype
    eps = np.ones(nt, dtype=dt_) if eps is None else np.asarray(eps, dtype=dt_)
    mu = np.ones(nt, dtype=dt_) if mu is None else np.asarray(mu, dtype=dt_)
    gg = np.einsum("tad,tbd->tab", g, g)      # g_a . g_b
    Te = np.zeros((nt, 6, 6), dtype=dt_)
    Se = np.zeros((nt, 6, 6), dtype=dt_)

    def m(a, b):                               # integral lam_a lam_b / V
        return dt_.type(2.0 if a == b else 1.0) / dt_.type(20.0)

    for A, (i, j) in enumerate(LOCAL_EDGES):
        cij = np.cross(g[:, i], g[:, j])
        for B, (k, l) in enumerate(LOCAL_EDGES):
            Te[:, A, B] = vol * (m(i, k) * gg[:, j, l] - m(i, l) * gg[:, j, k]
                                 - m(j, k) * gg[:, i, l] + m(j, l) * gg[:, i, k])
            ckl = np.cross(g[:, k], g[:, l])
            Se[:, A, B] = 4.0 * vol * np.einsum("td,td->t", cij, ckl)
    return Te * eps[:, None, None], Se / mu[:, None, None]


class Discretisation:
    """Edges, unknown numbering and assembled global matrices of one mesh."""

    def __init__(self, coords, tets, eps=None, mu=None, dtype=np.float64):
        self.dtype = np.dtype(dtype)
        self.coords = np.asarray(coords, dtype=self.dtype)
        self.tets = np.asarray(tets)
        self.edges, self.tet_edges = canonical_edges(self.tets)
        self.n_e = len(self.edges)
        self.pec = pec_mask(self.coords, self.edges)
        self.interior = np.flatnonzero(~self.pec)          # unknown -> edge
        self.n_int = len(self.interior)
        self.dof = np.full(self.n_e, -1, dtype=np.int64)   # edge -> unknown
        self.dof[self.interior] = np.arange(self.n_int)
        nt = len(self.tets)
        self.eps = np.ones(nt, self.dtype) if eps is None else np.asarray(eps, self.dtype)
        self.mu = np.ones(nt, self.dtype) if mu is None else np.asarray(mu, self.dtype)
        self.Te, self.Se = element_matrices(self.coords, self.tets, self.eps, self.mu)
        self.T = self._assemble(self.Te)
        self.S = self._assemble(self.Se)

    def _assemble(self, Ke):
        d = self.dof[self.tet_edges]                        # [n_t, 6]
        rows = np.repeat(d, 6, axis=1).ravel()
        cols = np.tile(d, (1, 6)).ravel()
        vals = Ke.reshape(len(d), 36).ravel()
        keep = (rows >= 0) & (cols >= 0)
        M = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])),
                          shape=(self.n_int, self.n_int)).tocsr()
        M.sum_duplicates()
        return M

    def unit_mass_elements(self):
        """Element mass matrices with eps = 1 (for the permittivity gradient)."""
        Te, _ = element_matrices(self.coords, self.tets)
        return Te

    # ---- vertices and the discrete gradient -------------------------------
    def interior_nodes(self):
        c = self.coords
        on = np.zeros(len(c), dtype=bool)
        for ax in range(3):
            on |= (c[:, ax] == 0.0) | (c[:, ax] == 1.0)
        return np.flatnonzero(~on)

    def gradient(self):
        """G [n_int edges, n_int nodes]: +1 at the head (higher id) of each
        edge, -1 at its tail, so that grad(phi_k) = sum_e G[e, k] W_e."""
        nodes = self.interior_nodes()
        nid = np.full(len(self.coords), -1, dtype=np.int64)
        nid[nodes] = np.arange(len(nodes))
        e = self.edges[self.interior]
        rows, cols, vals = [], [], []
        for end, sign in ((1, 1.0), (0, -1.0)):
            k = nid[e[:, end]]
            ok = k >= 0
            rows.append(np.flatnonzero(ok)); cols.append(k[ok])
            vals.append(np.full(ok.sum(), sign))
        return sp.csr_matrix((np.concatenate(vals),
                              (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.n_int, len(nodes)))

    # ---- conversions between full edge arrays and unknown vectors ----------
    def restrict(self, x_edges):
        """[..., n_e] -> [..., n_int]"""
        return np.asarray(x_edges)[..., self.interior]

    def extend(self, x_int):
        """[..., n_int] -> [..., n_e] with PEC entries 0."""
        x_int = np.asarray(x_int)
        out = np.zeros(x_int.shape[:-1] + (self.n_e,), dtype=x_int.dtype)
        out[..., self.interior] = x_int
        return out
