"""Write the oracle's gradient reference for the differentiation workload.

Calls only the oracle and the seeded input generators.  Workload: the 32^3
cavity (per-tet eps_r ~ U[1, 4] from seed 1, trainable), dt = 0.015, 50
Newmark steps, a trainable current J [50][200] on 200 seeded interior edges,
loss L = sum over 64 seeded probe edges of (e^50)^2.  The parameter vector
is theta = (eps [n_tets], J [50 * 200]) in that order; 20 directions d_k
from default_rng(5).standard_normal over theta, each normalised to unit
2-norm.

Stored (tests/golden/gradient_cavity32_box4_adjoint.npz):
  L0            the loss at theta
  fd[k]         (L(theta + h d_k) - L(theta - h d_k)) / (2h), h = 1e-6, each
                forward a fresh monolithic direct solve: the perturbed system
                assembled and the recurrence run in 80-bit extended precision,
                every step solved by the FP64 SuperLU factor refined on the
                extended residual (plain FP64 forwards leave a rounding floor
                of about 1e-14 L / h = 4e-10 here, up to 2.5e-5 of a
                directional derivative)
  fd_fp64[k]    the same differences with plain FP64 forwards (the floor)
  adj[k]        grad L . d_k from the oracle's reverse-mode adjoint
  jbar          dL/dJ [50, 200] (oracle adjoint)
  eps_idx, eps_bar_sample   4096 seeded tetrahedra and dL/deps there
  eps_bar_norm  |dL/deps|_2

Usage: python tests/golden/make_gradient_fixture.py [--workers 3] [--reuse-fp64]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.newmark import NewmarkOracle  # noqa: E402
from workloads.configs import workload  # noqa: E402
from workloads.sources import pulse  # noqa: E402

H = 1e-6
PATH = os.path.join(HERE, "gradient_cavity32_box4_adjoint.npz")


def problem():
    """(coords, tets, eps, src edges, probe edges, J amplitudes [N, 200],
    directions [20, n_tets + N*200], workload) of the differentiation case."""
    w = workload(4)
    ex = w.extra
    c, t = w.mesh()
    eps = w.eps(len(t))
    o = NewmarkOracle(c, t, dt=w.dt, factor=False)
    interior = o.d.interior
    src = interior[np.random.default_rng(ex["src_seed"]).choice(len(interior), ex["count"], replace=False)]
    probes = interior[np.random.default_rng(ex["probe_seed"]).choice(len(interior), ex["probes"], replace=False)]
    N = w.N
    amp = np.random.default_rng(ex["j_seed"]).uniform(-1, 1, (N, ex["count"])) * \
        pulse(N, w.dt, ex["t0"], ex["sigma"])[:, None]
    dirs = np.random.default_rng(ex["dir_seed"]).standard_normal((ex["dirs"], len(t) + amp.size))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    return c, t, eps, src, probes, amp, dirs, w


def loss(args):
    """L = sum_probes (e^N)^2 for (eps, amp) (FP64 direct solves, or the
    extended-precision recurrence: L then in longdouble), with the history
    if asked."""
    c, t, eps, src, probes, amp, dt, beta, n_e, keep, solver = args
    o = NewmarkOracle(c, t, eps=eps, dt=dt, beta=beta, solver=solver)
    J = np.zeros((amp.shape[0], 1, n_e), dtype=amp.dtype)
    J[:, 0, src] = amp
    E = o.run(J)
    L = np.sum(E[-1][0, probes] ** 2)
    return (float(L), o, J, E) if keep else L


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=3)
    ap.add_argument("--reuse-fp64", action="store_true",
                    help="take fd_fp64 from an existing file instead of recomputing it")
    a = ap.parse_args()
    c, t, eps, src, probes, amp, dirs, w = problem()
    n_t = len(t)
    n_e = NewmarkOracle(c, t, dt=w.dt, factor=False).d.n_e
    t0 = time.time()
    L0, o, J, E = loss((c, t, eps, src, probes, amp, w.dt, w.beta, n_e, True, "direct"))
    ebar = np.zeros_like(E[-1])
    ebar[0, probes] = 2.0 * E[-1][0, probes]
    Jbar, eps_bar = o.adjoint(J, E, ebar)
    jbar = Jbar[:, 0, src]
    grad = np.concatenate([eps_bar, jbar.ravel()])
    adj = dirs @ grad
    print(f"L0 {L0:.6e}, |grad| {np.linalg.norm(grad):.3e}, forward + adjoint {time.time() - t0:.0f} s",
          flush=True)
    import multiprocessing as mp
    fds = {}
    for solver in ("extended", "direct"):
        if solver == "direct" and a.reuse_fp64 and os.path.exists(PATH):
            old = np.load(PATH, allow_pickle=False)
            fds[solver] = old["fd_fp64"] if "fd_fp64" in old else old["fd"]
            continue
        ld = np.longdouble if solver == "extended" else np.float64
        h = ld(H)
        jobs = []
        for d in dirs:
            de, da = d[:n_t].astype(ld), d[n_t:].reshape(amp.shape).astype(ld)
            for sgn in (1, -1):
                jobs.append((c, t, eps.astype(ld) + sgn * h * de, src, probes, amp.astype(ld) + sgn * h * da,
                             w.dt, w.beta, n_e, False, solver))
        with mp.get_context("fork").Pool(a.workers) as pool:
            Ls = pool.map(loss, jobs, chunksize=1)
        Ls = np.array(Ls, dtype=ld).reshape(len(dirs), 2)
        fds[solver] = ((Ls[:, 0] - Ls[:, 1]) / (2 * h)).astype(np.float64)
        print(f"{solver} forwards done at {time.time() - t0:.0f} s", flush=True)
    fd, fd64 = fds["extended"], fds["direct"]
    for k in range(len(dirs)):
        print(f"direction {k}: fd {fd[k]:+.12e}  adjoint {adj[k]:+.12e}  "
              f"rel {abs(fd[k] - adj[k]) / max(abs(fd[k]), abs(adj[k])):.2e}  "
              f"(fp64 forwards: rel {abs(fd64[k] - adj[k]) / max(abs(fd64[k]), abs(adj[k])):.2e})", flush=True)
    idx = np.sort(np.random.default_rng(11).choice(n_t, 4096, replace=False))
    np.savez(PATH, L0=L0, h=H, fd=fd, fd_fp64=fd64, adj=adj, jbar=jbar, eps_idx=idx,
             eps_bar_sample=eps_bar[idx], eps_bar_norm=np.linalg.norm(eps_bar), workload=w.name)
    print(f"wrote {PATH} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
