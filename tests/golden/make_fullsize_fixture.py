"""Write the oracle's reference samples for the two full-size workloads.

Calls only the oracle and the seeded input generators.  For the 64^3 cavity
(1000 box subdomains, 16 beam right-hand sides) or the graded 48^3 cavity
(512 bisection subdomains, 32 right-hand sides) it runs the monolithic
Newmark recurrence (Sec. II-B-2), each step solved by Jacobi-preconditioned
conjugate gradients to a true relative residual of 1e-13 with a certified
error bound, and stores for every step n = 1..N and right-hand side r:

  norm[n-1, r]        |e^n_r|_2 over all canonical edges
  idx[n-1, :]         sampled interior edges (workloads.probes.sample_edges)
  val[n-1, r, :]      e^n_r on those edges
  sketch[n-1, r, k]   g_k . e^n_r, g_k = workloads.probes.sketch_vectors rows
  gauss[n-1, r]       max over interior vertices of |G^T T e^n + q^n|
  qmax[n-1, r]        max |q^n|
  log[n-1, :]         PCG iterations, true relative residual, error bound

Usage: python tests/golden/make_fullsize_fixture.py cavity64|graded48
           [--steps 25] [--workers 8]
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
from workloads.probes import sample_edges, sketch_vectors  # noqa: E402

CASES = {
    # workload index, sampled edges per step (shared by the RHS)
    "cavity64": (5, 256),
    "graded48": (3, 128),
}
SAMPLE_SEED = 77
SKETCH_SEED = 78
SKETCHES = 16


def fixture_path(name):
    return os.path.join(HERE, f"fullsize_{workload(CASES[name][0]).name}.npz")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=sorted(CASES))
    ap.add_argument("--steps", type=int, default=25)
    ap.add_argument("--workers", type=int, default=8)
    a = ap.parse_args()
    k, m = CASES[a.case]
    w = workload(k)
    N = a.steps
    log = lambda *x: print(f"[{a.case}]", *x, flush=True)
    c, t = w.mesh()
    t0 = time.time()
    J = w.sources_for_steps(t, c, range(N), workers=a.workers)          # [N, nrhs, n_e]
    log(f"sources {J.shape} in {time.time() - t0:.0f} s")
    t0 = time.time()
    o = NewmarkOracle(c, t, eps=w.eps(len(t)), dt=w.dt, beta=w.beta, solver="pcg", pcg_tol=1e-13)
    d = o.d
    G = d.gradient()
    log(f"assembly in {time.time() - t0:.0f} s; n_int {d.n_int}, lambda_lo {o.lam_lo:.3e}")
    Gk = sketch_vectors(d.n_e, SKETCHES, SKETCH_SEED)
    nr = w.nrhs
    out = {k2: [] for k2 in ("norm", "idx", "val", "sketch", "gauss", "qmax", "log")}
    e_nm1 = np.zeros((nr, d.n_int))
    e_n = np.zeros((nr, d.n_int))
    j_prev = np.zeros((nr, d.n_int))
    q = np.zeros((nr, G.shape[1]))
    for n in range(N):
        t0 = time.time()
        jn = d.restrict(J[n])
        e = o.step(e_n, e_nm1, jn, j_prev)
        q = q + o.dt * (G.T @ jn.T).T
        gauss = np.abs((G.T @ (d.T @ e.T)).T + q).max(axis=1)
        full = d.extend(e)
        idx = sample_edges(d.interior, n + 1, m, SAMPLE_SEED)
        out["norm"].append(np.linalg.norm(full, axis=1))
        out["idx"].append(idx)
        out["val"].append(full[:, idx])
        out["sketch"].append(full @ Gk.T)
        out["gauss"].append(gauss)
        out["qmax"].append(np.abs(q).max(axis=1))
        it, rel, bound = o.solve_log[-1]
        out["log"].append((it, rel, bound))
        log(f"step {n + 1}: {it} PCG iterations, relres {rel:.2e}, error bound {bound:.2e}, "
            f"Gauss {gauss.max():.2e} (max |q| {out['qmax'][-1].max():.2e}), {time.time() - t0:.0f} s")
        e_nm1, e_n, j_prev = e_n, e, jn
    arrays = {k2: np.asarray(v) for k2, v in out.items()}
    np.savez(fixture_path(a.case), workload=w.name, steps=N, sample_seed=SAMPLE_SEED,
             sketch_seed=SKETCH_SEED, sketches=SKETCHES, n_edges=d.n_e, **arrays)
    log(f"wrote {fixture_path(a.case)}")


if __name__ == "__main__":
    main()
