"""Reverse-mode differentiation of the Newmark field update.

NewmarkDD.apply(J, eps, solver, checkpoint_every) -> E^N

  J    [N, nrhs, n_edges] float64 device tensor: J^{n+1/2}, n = 0..N-1
  eps  [n_tets] float64 tensor (relative permittivity per tetrahedron)
  returns e^N [nrhs, n_edges] (e^0 = e^-1 = 0, J^{-1/2} = 0)

Forward keeps only (e^m, e^{m-1}) at every checkpoint_every-th step.  The
backward pass replays each segment forward from its checkpoint and runs the
hand-written adjoint step of the library (dd_adjoint_step, which reuses the
symmetric factors and accumulates every gradient itself):
    g^n = A^-1 ebar^{n+1};  ebar^n += (2A - dt^2 S) g^n;  ebar^{n-1} -= A g^n;
    eps_bar_k -= g^n . T_k (e^{n+1} - 2 e^n + e^{n-1});
    Jbar^{n+1/2} += -dt g^n,  Jbar^{n-1/2} += dt g^n.
This module only orders the calls (checkpoints, replays, buffers).
"""
from __future__ import annotations

import numpy as np
import torch


def _set_eps(solver, eps):
    e = eps.detach().to("cpu", torch.float64).numpy()
    if getattr(solver, "_eps_cache", None) is None or not np.array_equal(solver._eps_cache, e):
        solver.set_eps(e)
        solver.factor()
        solver._eps_cache = e.copy()


def _forward_steps(solver, J, E_nm1, E_n, J_prev, n0, n1, keep=None):
    """Advance from (e^{n0-1}, e^{n0}) through steps n0..n1-1; returns the
    last two states, and appends every e^{n+1} to keep if given."""
    for n in range(n0, n1):
        E_next = solver.step(J[n], J_prev, E_n, E_nm1)
        if keep is not None:
            keep.append(E_next)
        E_nm1, E_n, J_prev = E_n, E_next, J[n]
    return E_nm1, E_n


class NewmarkDD(torch.autograd.Function):
    @staticmethod
    def forward(ctx, J, eps, solver, checkpoint_every=10):
        _set_eps(solver, eps)
        N = J.shape[0]
        k = max(1, int(checkpoint_every))
        zero = torch.zeros_like(J[0])
        E_nm1, E_n = zero, zero.clone()
        ckpt = {0: (E_nm1, E_n)}
        for m in range(0, N, k):
            E_nm1, E_n = _forward_steps(solver, J, E_nm1, E_n, J[m - 1] if m > 0 else zero, m, min(N, m + k))
            if m + k < N:
                ckpt[m + k] = (E_nm1.clone(), E_n.clone())
        ctx.solver = solver
        ctx.k = k
        ctx.ckpt = ckpt
        ctx.save_for_backward(J, eps)
        return E_n.clone()

    @staticmethod
    def backward(ctx, gE):
        J, eps = ctx.saved_tensors
        s, k = ctx.solver, ctx.k
        _set_eps(s, eps)
        N = J.shape[0]
        zero = torch.zeros_like(J[0])
        eps_bar = torch.zeros(s.n_tets, dtype=torch.float64, device=J.device)
        Jbar = torch.zeros_like(J)
        g_buf = torch.empty_like(zero)
        # ebar buffers for the current window: ebar[n] accumulates until step n-1 is processed
        ebar = {N: gE.contiguous().clone(), N - 1: zero.clone()}
        starts = list(range(0, N, k))
        for m in reversed(starts):
            m1 = min(N, m + k)
            E_nm1, E_n = ctx.ckpt[m]
            hist = [E_nm1, E_n]                    # e^{m-1}, e^m, then e^{m+1}..e^{m1}
            _forward_steps(s, J, E_nm1, E_n, J[m - 1] if m > 0 else zero, m, m1, keep=hist)
            for n in range(m1 - 1, m - 1, -1):
                if n - 1 not in ebar:
                    ebar[n - 1] = zero.clone()
                e_next, e_n = hist[n + 1 - m + 1], hist[n - m + 1]
                e_nm1 = hist[n - m] if n >= 1 else None
                s.adjoint_step(ebar[n + 1], ebar[n], ebar[n - 1] if n >= 1 else None,
                               e_next, e_n, e_nm1, eps_bar, g_out=g_buf,
                               Jbar_half=Jbar[n], Jbar_prev_half=Jbar[n - 1] if n >= 1 else None)
                del ebar[n + 1]
        return Jbar, eps_bar.to(eps.device, eps.dtype), None, None
