"""Thin Python front-end over the C ABI: torch tensors provide device memory
and the stream; the library does all the work."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import DD_FP32_REFINE, DD_FP64, Analysis, Info, Mesh, Options, Stats, Tuning, check, load


def _host(a, dtype):
    a = np.ascontiguousarray(np.asarray(a), dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _dev(t: torch.Tensor):
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 device tensor")
    return C.c_void_p(t.data_ptr())


def _dev_i32(t: torch.Tensor):
    if t.device.type != "cuda" or t.dtype != torch.int32 or not t.is_contiguous():
        raise ValueError("expected a contiguous int32 device tensor")
    return C.c_void_p(t.data_ptr())


def _mesh(coords, tets):
    """dd_mesh over contiguous host copies (returned to keep them alive)."""
    c, cp = _host(coords, np.float64)
    t, tp = _host(tets, np.int32)
    return Mesh(len(c), cp, len(t), tp), (c, t)


def analyze(coords, tets, partition):
    """Host-only partition analysis: (Analysis, per_sub [n_sub, 3])."""
    lib = load()
    m, keep = _mesh(coords, tets)
    p, pp = _host(partition, np.int32)
    out = Analysis()
    check(lib.dd_analyze(C.byref(m), pp, C.byref(out), None))
    per = np.zeros((out.n_sub, 3), dtype=np.int32)
    check(lib.dd_analyze(C.byref(m), pp, C.byref(out), per.ctypes.data_as(C.c_void_p)))
    return out, per


def analyze_lambda(coords, tets, partition, n_lambda):
    lib = load()
    m, keep = _mesh(coords, tets)
    p, pp = _host(partition, np.int32)
    arrs = [np.zeros(n_lambda, dtype=np.int32) for _ in range(5)]
    check(lib.dd_analyze_lambda(C.byref(m), pp, *[a.ctypes.data_as(C.c_void_p) for a in arrs]))
    return dict(zip(("edge", "sub_lo", "sub_hi", "pos_lo", "pos_hi"), arrs))


class DDSolver:
    """Decomposed Newmark solver on one GPU.

    Arrays crossing the boundary: fields and currents are float64 device
    tensors [nrhs, n_edges] on canonical edges.
    """

    def __init__(self, coords, tets, partition, eps, mu=None, dt=0.05, beta=0.25, *,
                 precision="fp64", nrhs=1, cg_tol=1e-10, cg_max_iter=500, refine_tol=1e-12,
                 refine_max=10, warm_start=0, check_every=4, stream=None, factor=True,
                 use_graph=False, precond=1, method="dp1", robin_alpha=0.0, diagnostics=0,
                 tune_cache=None):
        self.lib = load()
        o = Options()
        self.lib.dd_default_options(C.byref(o))
        o.precision = DD_FP32_REFINE if precision == "fp32_refine" else DD_FP64
        o.nrhs = int(nrhs)
        o.cg_tol = float(cg_tol)
        o.cg_max_iter = int(cg_max_iter)
        o.refine_tol = float(refine_tol)
        o.refine_max = int(refine_max)
        o.warm_start = int(warm_start)
        o.check_every = int(check_every)
        o.use_graph = int(bool(use_graph))
        o.precond = int(precond)
        if method not in ("dp1", "dp2"):
            raise ValueError("method must be 'dp1' or 'dp2'")
        o.method = 1 if method == "dp2" else 0
        o.robin_alpha = float(robin_alpha)
        o.diagnostics = int(diagnostics)
        o.tune_cache = None if tune_cache is None else str(tune_cache).encode()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        o.stream = C.c_void_p(stream.cuda_stream)
        self.opt = o
        mesh, keep = _mesh(coords, tets)
        p, pp = _host(partition, np.int32)
        e, ep = _host(eps, np.float64)
        mp = None
        if mu is not None:
            m, mp = _host(mu, np.float64)
        h = C.c_void_p()
        check(self.lib.dd_setup(C.byref(h), C.byref(mesh), pp, ep, mp, float(dt), float(beta), C.byref(o)))
        self.h = h
        self.nrhs = int(nrhs)
        self.dt = float(dt)
        inf = self.info
        self.n_edges = inf.n_edges
        self.n_tets = inf.n_tets
        self.n_vertices = inf.n_vertices
        self.stats = Stats()
        if factor:
            self.factor()

    @property
    def info(self):
        """Sizes and byte counts (the coarse byte count reflects the stored
        nonzero tiles once the context is factorised)."""
        inf = Info()
        check(self.lib.dd_get_info(self.h, C.byref(inf)))
        return inf

    # ---- lifecycle -----------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.dd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- calls ------------------------------------------------------------------------
    def edges(self):
        e = np.zeros((self.n_edges, 2), dtype=np.int32)
        pec = np.zeros(self.n_edges, dtype=np.uint8)
        check(self.lib.dd_get_edges(self.h, e.ctypes.data_as(C.c_void_p),
                                    pec.ctypes.data_as(C.c_void_p)))
        return e, pec.astype(bool)

    def set_eps(self, eps):
        """eps: host array, or a float64 device tensor (validated by the
        library on the host either way)."""
        if isinstance(eps, torch.Tensor) and eps.device.type == "cuda":
            check(self.lib.dd_set_eps(self.h, _dev(eps), 1))
        else:
            e, ep = _host(eps, np.float64)
            check(self.lib.dd_set_eps(self.h, ep, 0))

    def set_charge(self, q=None):
        """Accumulated nodal charge of the per-step Gauss check: device
        tensor [nrhs, n_vertices], or None for zero."""
        check(self.lib.dd_set_charge(self.h, None if q is None else _dev(q)))

    def factor(self):
        check(self.lib.dd_factor(self.h))

    def autotune(self, cache=None):
        """Tune the work-list shapes (dd_autotune); returns them and the
        measured times as a dict."""
        t = Tuning()
        check(self.lib.dd_autotune(self.h, None if cache is None else str(cache).encode(), C.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def new_field(self):
        return torch.zeros((self.nrhs, self.n_edges), dtype=torch.float64, device="cuda")

    def step(self, J_half, J_prev_half, E_n, E_nm1, E_next=None, stats=False, raise_on_error=True):
        if E_next is None:
            E_next = self.new_field()
        rc = self.lib.dd_step(self.h, _dev(J_half), _dev(J_prev_half), _dev(E_n), _dev(E_nm1),
                              _dev(E_next), C.byref(self.stats) if stats else None)
        if raise_on_error:
            check(rc)
        return E_next

    def solve(self, b, x=None, stats=True):
        if x is None:
            x = self.new_field()
        check(self.lib.dd_solve(self.h, _dev(b), _dev(x), C.byref(self.stats) if stats else None))
        return x

    def adjoint_step(self, ebar_next, ebar_n, ebar_nm1, E_next, E_n, E_nm1, eps_bar, g_out=None,
                     Jbar_half=None, Jbar_prev_half=None):
        """One reverse step (dd_adjoint_step); the library accumulates
        -dt g into Jbar_half and +dt g into Jbar_prev_half when given."""
        if g_out is None:
            g_out = self.new_field()
        p = lambda t: None if t is None else _dev(t)
        check(self.lib.dd_adjoint_step(self.h, _dev(ebar_next), p(ebar_n), p(ebar_nm1), _dev(g_out),
                                       p(E_next), p(E_n), p(E_nm1), p(eps_bar), p(Jbar_half),
                                       p(Jbar_prev_half), None))
        return g_out

    def charge_update(self, J_half, q):
        check(self.lib.dd_charge_update(self.h, _dev(J_half), _dev(q)))

    def gauss_residual(self, E, q):
        out = np.zeros(self.nrhs)
        check(self.lib.dd_gauss_residual(self.h, _dev(E), _dev(q), out.ctypes.data_as(C.c_void_p)))
        return out

    def energy(self, E_next, E_n):
        out = np.zeros(self.nrhs)
        check(self.lib.dd_energy(self.h, _dev(E_next), _dev(E_n), out.ctypes.data_as(C.c_void_p)))
        return out

    # ---- mixed E/B step (dd_step_mixed) ------------------------------------------
    def faces(self):
        """Canonical faces [n_faces, 3] (host int32)."""
        nf = C.c_int64(0)
        check(self.lib.dd_mixed_faces(self.h, C.byref(nf), None))
        f = np.zeros((nf.value, 3), dtype=np.int32)
        check(self.lib.dd_mixed_faces(self.h, None, f.ctypes.data_as(C.c_void_p)))
        self.n_faces = nf.value
        return f

    def new_face_field(self):
        if not hasattr(self, "n_faces"):
            self.faces()
        return torch.zeros((self.nrhs, self.n_faces), dtype=torch.float64, device="cuda")

    def step_mixed(self, J_half, E_n, B_n, E_next=None, B_next=None, stats=False):
        """One trapezoid step of the mixed E/B system; returns (E_next, B_next)."""
        if not hasattr(self, "n_faces"):
            self.faces()
        E_next = self.new_field() if E_next is None else E_next
        B_next = self.new_face_field() if B_next is None else B_next
        for t, n in ((J_half, self.n_edges), (E_n, self.n_edges), (E_next, self.n_edges)):
            self._len(t, self.nrhs * n, "edge array")
        for t in (B_n, B_next):
            self._len(t, self.nrhs * self.n_faces, "face array")
        check(self.lib.dd_step_mixed(self.h, _dev(J_half), _dev(E_n), _dev(B_n), _dev(E_next), _dev(B_next),
                                     C.byref(self.stats) if stats else None))
        return E_next, B_next

    # ---- particle steps (dd_pic_*): device tensors, positions [n, 3] ----------
    @staticmethod
    def _pts(x, n=None):
        if x.dim() != 2 or x.shape[1] != 3 or (n is not None and x.shape[0] != n):
            raise ValueError("expected positions / velocities of shape [n, 3]")
        return x.shape[0]

    @staticmethod
    def _len(t, n, name):
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} entries, expected {n}")

    PIC_COUNTERS = ("absorbed_or_outside", "walk_cap", "bad_index")

    def pic_status(self, reset=True):
        """Device counters of the particle calls since the last reset (syncs)."""
        c = np.zeros(3, dtype=np.int64)
        check(self.lib.dd_pic_status(self.h, c.ctypes.data_as(C.c_void_p), int(bool(reset))))
        return dict(zip(self.PIC_COUNTERS, (int(v) for v in c)))

    def pic_locate(self, x, cell=None):
        """Containing tetrahedron of each point (walk from cell, default 0);
        points outside the mesh get -1 (counted in pic_status)."""
        n = self._pts(x)
        if cell is None:
            cell = torch.zeros(n, dtype=torch.int32, device=x.device)
        self._len(cell, n, "cell")
        check(self.lib.dd_pic_locate(self.h, n, _dev(x), _dev_i32(cell)))
        return cell

    def pic_deposit(self, xa, xb, q, cell, J):
        """J += exact edge currents of the paths xa -> xb (J: one row
        [n_edges]); cell is advanced to the end points (-1 for particles
        absorbed at the outer boundary, counted in pic_status)."""
        n = self._pts(xa)
        self._pts(xb, n)
        self._len(q, n, "q")
        self._len(cell, n, "cell")
        self._len(J, self.n_edges, "J")
        check(self.lib.dd_pic_deposit(self.h, n, _dev(xa), _dev(xb), _dev(q), _dev_i32(cell), _dev(J)))

    def pic_sort(self, cell):
        """Permutation [n] int32 that orders the particles by cell."""
        n = cell.numel()
        perm = torch.empty(n, dtype=torch.int32, device=cell.device)
        check(self.lib.dd_pic_sort(self.h, n, _dev_i32(cell), _dev_i32(perm)))
        return perm

    def pic_sort_noalloc(self, cell, perm):
        """pic_sort through the allocation-free entry point (the caller
        provides perm [n] int32; the library's static scratch serves the
        counts)."""
        n = cell.numel()
        self._len(perm, n, "perm")
        check(self.lib.dd_pic_sort_noalloc(self.h, n, _dev_i32(cell), _dev_i32(perm)))
        return perm

    def pic_permute(self, perm, src, dst=None):
        """dst[i] = src[perm[i]] along the first axis (any dtype, contiguous)."""
        n = perm.numel()
        if not src.is_contiguous() or src.shape[0] != n or src.device.type != "cuda":
            raise ValueError("src must be a contiguous device tensor with perm.numel() rows")
        if dst is None:
            dst = torch.empty_like(src)
        if dst.shape != src.shape or dst.dtype != src.dtype or not dst.is_contiguous():
            raise ValueError("dst must match src")
        item = src.element_size() * (src.numel() // max(n, 1))
        check(self.lib.dd_pic_permute(self.h, n, _dev_i32(perm), item, C.c_void_p(src.data_ptr()),
                                      C.c_void_p(dst.data_ptr())))
        return dst

    def pic_faraday(self, E, alpha, B):
        """B += alpha * curl E per tetrahedron; E [n_edges] or [r, n_edges],
        B [n_tets, 3] or [r, n_tets, 3]."""
        rows = E.numel() // self.n_edges
        self._len(E, rows * self.n_edges, "E")
        self._len(B, 3 * rows * self.n_tets, "B")
        check(self.lib.dd_pic_faraday(self.h, rows, _dev(E), float(alpha), _dev(B)))

    def pic_push(self, qm, E, B, cell, x, x_new, v, hist, first):
        """Interpolate E, B at x and take one Adams-Bashforth step (x_new, v,
        hist updated in place)."""
        n = self._pts(x)
        self._pts(x_new, n)
        self._pts(v, n)
        self._len(qm, n, "qm")
        self._len(cell, n, "cell")
        self._len(hist, 6 * n, "hist")
        self._len(E, self.n_edges, "E")
        self._len(B, 3 * self.n_tets, "B")
        check(self.lib.dd_pic_push(self.h, x.shape[0], _dev(qm), _dev(E), _dev(B), _dev_i32(cell), _dev(x),
                                   _dev(x_new), _dev(v), _dev(hist), 1 if first else 0))

    PROF_CLASSES = ("trailing", "full", "schur", "coarse", "corner", "cross")

    def profile(self, enable=-1):
        """Per-class (ms, launches) of the tile products since the last reset;
        enable=1/0 turns event timing on/off and resets."""
        ms = np.zeros(len(self.PROF_CLASSES))
        n = np.zeros(len(self.PROF_CLASSES), dtype=np.int64)
        check(self.lib.dd_profile(self.h, int(enable), ms.ctypes.data_as(C.c_void_p),
                                  n.ctypes.data_as(C.c_void_p)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.PROF_CLASSES)}

    def state_set(self, E_n=None, E_nm1=None, J_prev_half=None):
        """Load the context's resident Newmark state (dd_state_set); None is
        zero."""
        for a, nm in ((E_n, "E_n"), (E_nm1, "E_nm1"), (J_prev_half, "J_prev_half")):
            if a is not None:
                self._len(a, self.nrhs * self.n_edges, nm)
        check(self.lib.dd_state_set(self.h, None if E_n is None else _dev(E_n),
                                    None if E_nm1 is None else _dev(E_nm1),
                                    None if J_prev_half is None else _dev(J_prev_half)))

    def step_resident(self, J_half, E_next=None, stats=False, raise_on_error=True):
        """One Newmark step of the resident state (dd_step_resident)."""
        if E_next is None:
            E_next = self.new_field()
        self._len(J_half, self.nrhs * self.n_edges, "J_half")
        self._len(E_next, self.nrhs * self.n_edges, "E_next")
        rc = self.lib.dd_step_resident(self.h, _dev(J_half), _dev(E_next), C.byref(self.stats) if stats else None)
        if raise_on_error:
            check(rc)
        return E_next

    def last_stats(self):
        s = self.stats
        n = self.nrhs
        d = dict(cg_iters=list(s.cg_iters[:n]), refine_sweeps=s.refine_sweeps,
                 dd_solves=s.dd_solves, cg_relres=list(s.cg_relres[:n]),
                 global_relres=list(s.global_relres[:n]), solve_iters=list(s.solve_iters),
                 diagnostics=s.diagnostics)
        if s.diagnostics & 1:
            d["gauss_residual"] = list(s.gauss_residual[:n])
            d["charge_max"] = list(s.charge_max[:n])
        if s.diagnostics & 2:
            d["energy"] = list(s.energy[:n])
        return d
