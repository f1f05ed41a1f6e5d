"""The five seeded workloads (sizes, partitions, materials, time steps,
sources, solver settings).  Pure input description: no solver arithmetic.

Where the workload statements leave a value open (pulse shape, source and
probe edges, time step of the larger cases) the value chosen here is the one
recorded in the design notes; every random draw is seeded with
numpy.random.default_rng, one vectorised draw per quantity.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import mesh as _mesh
from . import partition as _part
from . import sources as _src


@dataclass
class Workload:
    name: str
    n: int
    grade: float
    parts: object                 # (px, py, pz) boxes, or ("rcb", levels, seed)
    dt: float
    N: int
    nrhs: int
    precision: str                # "fp64" or "fp32_refine"
    cg_tol: float
    check_tol: float
    eps_seed: int | None = None   # eps_r ~ U[1, 4] per tet from this seed
    refine_tol: float = 1e-12
    beta: float = 0.25
    extra: dict = field(default_factory=dict)

    def mesh(self):
        c, t, _ = _mesh.cube_mesh(self.n, self.grade)
        return c, t

    def partition(self):
        if isinstance(self.parts, tuple) and self.parts and self.parts[0] == "rcb":
            return _part.rcb_partition(self.n, self.parts[1], self.parts[2])
        return _part.box_partition(self.n, self.parts)

    def eps(self, n_t):
        if self.eps_seed is None:
            return np.ones(n_t)
        return np.random.default_rng(self.eps_seed).uniform(1.0, 4.0, n_t)

    def mu(self, n_t):
        return np.ones(n_t)

    def sources_for_steps(self, tets, coords, steps, workers=1, start_method="fork"):
        """J_half [len(steps), nrhs, n_e] for the given step indices.  Beam
        currents (one deposit of every particle path per step and RHS) are
        spread over `workers` processes, one right-hand side per task; use
        start_method="spawn" in a process that has initialised a GPU."""
        steps = list(steps)
        if self.extra.get("source") != "beam":
            return self.sources(tets, coords, N=max(steps) + 1)[steps]
        edges = _mesh.mesh_edges(tets)
        jobs = [(coords, tets, edges, self.n, self.dt, self.extra["beam"], r, steps)
                for r in range(self.nrhs)]
        if workers > 1:
            import multiprocessing as mp
            with mp.get_context(start_method).Pool(min(workers, len(jobs))) as pool:
                parts = pool.map(_beam_rhs, jobs)
        else:
            parts = [_beam_rhs(j) for j in jobs]
        return np.stack(parts, axis=1)

    def sources(self, tets, coords, N=None):
        """J_half [N, nrhs, n_e] for the first N steps (default: all)."""
        N = self.N if N is None else N
        edges = _mesh.mesh_edges(tets)
        interior = ~_mesh.boundary_edge_mask(coords, edges)
        ex = self.extra
        kind = ex.get("source", "dense")
        if kind == "dense":
            return _src.dense_random_source(len(edges), interior, N, self.dt,
                                            ex["t0"], ex["sigma"], ex["seed"],
                                            nrhs=self.nrhs)
        if kind == "sparse":
            return _src.sparse_random_source(len(edges), interior, N, self.dt,
                                             ex["t0"], ex["sigma"], ex["seed"],
                                             ex["count"])
        if kind == "beam":
            from . import beam
            return beam.beam_source(coords, tets, edges, self.n, N, self.dt,
                                    self.nrhs, **ex["beam"])
        raise ValueError(kind)


def _beam_rhs(args):
    """Beam currents of one right-hand side (a process-pool task)."""
    coords, tets, edges, n, dt, beam, r, steps = args
    from .beam import beam_source
    b = dict(beam)
    b["seed"] = beam["seed"] + r
    return beam_source(coords, tets, edges, n, 0, dt, 1, steps=steps, **b)[:, 0, :]


def workload(k: int) -> Workload:
    if k == 1:
        N, dt = 10, 0.05
        return Workload("cavity8_box2", 8, 1.0, (2, 2, 2), dt, N, 1, "fp64", 1e-12, 1e-10,
                        extra=dict(source="dense", seed=0, t0=N * dt / 2, sigma=N * dt / 8))
    if k == 2:
        # CG tol 1e-13: with 1e-10 the per-step solve error (2e-11) grows
        # quadratically in the step count to 1.2e-8 by step 100
        return Workload("cavity24_box4_eps", 24, 1.0, (4, 4, 4), 0.02, 100, 1, "fp64",
                        1e-13, 1e-10, eps_seed=1,
                        extra=dict(source="sparse", seed=2, count=1000, t0=1.0, sigma=0.25))
    if k == 3:
        return Workload("graded48_rcb512_32rhs", 48, 1.5, ("rcb", 9, 0), 0.01, 50, 32,
                        "fp32_refine", 1e-6, 1e-8,
                        extra=dict(source="dense", seed=100, t0=0.25, sigma=0.0625))
    if k == 4:
        return Workload("cavity32_box4_adjoint", 32, 1.0, (4, 4, 4), 0.015, 50, 1, "fp64",
                        1e-12, 1e-10, eps_seed=1,
                        extra=dict(source="sparse_trainable", src_seed=2, count=200,
                                   j_seed=3, t0=0.375, sigma=0.094, probe_seed=4,
                                   probes=64, dir_seed=5, dirs=20, checkpoint=10))
    if k == 5:
        return Workload("cavity64_box10_beam16", 64, 1.0, (10, 10, 10), 0.008, 200, 16,
                        "fp32_refine", 1e-6, 1e-8,
                        extra=dict(source="beam",
                                   beam=dict(particles=1_000_000, radius=0.2, vth=0.01,
                                             vz=0.3, q0=1e-6, seed=1000)))
    raise ValueError(k)
