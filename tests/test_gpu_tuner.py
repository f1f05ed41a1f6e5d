"""The work-list autotuner (dd_autotune): a timed search on an uneven
partition, its JSON-lines cache (written, read back by a second context,
applied without timing), and parity with the oracle on tuned and on
deliberately odd shapes (split rows, short chunks, no placement buckets),
with the captured CG graph rebuilt after every change of the lists."""
import json

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


def _steps(s, J):
    N, nrhs, ne = J.shape
    Jd = torch.tensor(J, device="cuda")
    z = torch.zeros((nrhs, ne), dtype=torch.float64, device="cuda")
    E = [z, z.clone()]
    for n in range(N):
        E.append(s.step(Jd[n], Jd[n - 1] if n else z, E[-1], E[-2], stats=True))
    return torch.stack(E[2:]).cpu().numpy()


def _err(E, Eo):
    return max(np.linalg.norm(E[k] - Eo[k + 1], axis=1).max() / np.linalg.norm(Eo[k + 1], axis=1).max()
               for k in range(len(E)))


def test_tuner_search_cache_and_parity(tmp_path):
    from paper_2204_13254_amd.solver import DDSolver
    c, t, p, eps = _case()
    dt = 0.03
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    J = dense_random_source(o.d.n_e, ~o.d.pec, 4, dt, 0.06, 0.03, seed=5, nrhs=16)
    Eo = o.run(J)
    cache = tmp_path / "tune.jsonl"
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = DDSolver(c, t, p, eps, dt=dt, precision="fp32_refine", nrhs=16, cg_tol=1e-6, stream=st,
                     use_graph=True)
        E0 = _steps(s, J)                       # default shapes, graph captured
        r = s.autotune(cache)
        print("tuned", r, flush=True)
        assert r["from_cache"] == 0
        assert r["full_ms"] <= r["full_ms_default"] and r["trailing_ms"] <= r["trailing_ms_default"]
        E1 = _steps(s, J)                       # tuned shapes, graph recaptured
    st.synchronize()
    assert _err(E0, Eo) <= 1e-8 and _err(E1, Eo) <= 1e-8
    lines = [json.loads(x) for x in cache.read_text().splitlines()]
    assert len(lines) == 1 and lines[0]["full_chunk"] == r["full_chunk"]
    # a second context reads the cache (no timing) through the option
    with torch.cuda.stream(st):
        s2 = DDSolver(c, t, p, eps, dt=dt, precision="fp32_refine", nrhs=16, cg_tol=1e-6, stream=st,
                      use_graph=True, tune_cache=str(cache))
        r2 = s2.autotune(cache)
        E2 = _steps(s2, J)
    st.synchronize()
    assert r2["from_cache"] == 1
    assert all(r2[k] == r[k] for k in ("chunk", "coarse_chunk", "full_chunk", "full_bucket"))
    assert _err(E2, Eo) <= 1e-8


def test_odd_shapes_from_cache_keep_parity(tmp_path):
    """Short chunks split almost every row into partial slots (reduced in a
    fixed order), in every product class, a 16-workgroup persistent grid
    walks all work groups of the full passes, and an 8-workgroup one all
    panel pairs of the symmetric product."""
    from paper_2204_13254_amd.solver import DDSolver
    c, t, p, eps = _case()
    dt = 0.03
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    J = dense_random_source(o.d.n_e, ~o.d.pec, 3, dt, 0.05, 0.03, seed=9, nrhs=3)
    Eo = o.run(J)
    s = DDSolver(c, t, p, eps, dt=dt, precision="fp64", nrhs=3, cg_tol=1e-12)
    probe = tmp_path / "probe.jsonl"
    s.autotune(probe)                            # writes this context's key
    key = json.loads(probe.read_text().splitlines()[0])["key"]
    odd = tmp_path / "odd.jsonl"
    odd.write_text(json.dumps({"key": key, "chunk": 2, "coarse_chunk": 3, "full_chunk": 4,
                               "full_bucket": 1, "full_persist": 16, "sym_persist": 8}) + "\n")
    r = s.autotune(odd)
    assert r["from_cache"] == 1 and (r["chunk"], r["full_chunk"], r["full_persist"]) == (2, 4, 16)
    assert r["sym_persist"] == 8
    assert _err(_steps(s, J), Eo) <= 1e-10


@pytest.mark.parametrize("pair,chunk,persist,quarter", [(1, 3, 0, 1), (1, 96, 0, 1), (2, 96, 0, 1), (2, 96, 16, 1),
                                                        (0, 96, 0, 0), (0, 5, 0, 1), (1, 96, 0, 0)])
def test_row_pair_full_passes(tmp_path, pair, chunk, persist, quarter):
    """Two output rows per wave (pair 1) or eight rows per workgroup sharing
    each input block through LDS (pair 2) over the union of their tile lists
    (absent tiles read from a zero tile); pairs split into 3-entry chunks or
    whole, octets on a 16-workgroup persistent grid too; all-zero tile
    quarters read from the zero tile or from memory; with 16 and 24
    right-hand sides (one and two 16-wide MFMA blocks)."""
    from paper_2204_13254_amd.solver import DDSolver
    c, t, p, eps = _case()
    dt = 0.03
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    for nrhs, prec, tol in ((16, "fp32_refine", 1e-8), (24, "fp64", 1e-10)):
        J = dense_random_source(o.d.n_e, ~o.d.pec, 3, dt, 0.05, 0.03, seed=13, nrhs=nrhs)
        Eo = o.run(J)
        s = DDSolver(c, t, p, eps, dt=dt, precision=prec, nrhs=nrhs, cg_tol=1e-6 if prec != "fp64" else 1e-12)
        probe = tmp_path / f"probe{nrhs}.jsonl"
        s.autotune(probe)
        key = json.loads(probe.read_text().splitlines()[0])["key"]
        f = tmp_path / f"pair{nrhs}.jsonl"
        f.write_text(json.dumps({"key": key, "chunk": 32, "coarse_chunk": 16, "full_chunk": chunk,
                                 "full_bucket": 8, "full_pair": pair, "full_persist": persist,
                                 "full_quarter": quarter}) + "\n")
        r = s.autotune(f)
        assert (r["full_pair"], r["full_persist"], r["full_quarter"]) == (pair, persist, quarter)
        assert _err(_steps(s, J), Eo) <= tol, (nrhs, chunk)


def test_symmetric_product_shapes(tmp_path):
    """The interface operator's symmetric product with panels of two
    interface blocks (twice the partial slots) on a 16-workgroup persistent
    grid, with 16 and 24 right-hand sides (one and two 16-wide MFMA blocks),
    FP32 factors with refinement, against the oracle."""
    from paper_2204_13254_amd.solver import DDSolver
    c, t, p, eps = _case()
    dt = 0.03
    o = NewmarkOracle(c, t, eps=eps, dt=dt)
    for nrhs in (16, 24):
        J = dense_random_source(o.d.n_e, ~o.d.pec, 3, dt, 0.05, 0.03, seed=17, nrhs=nrhs)
        Eo = o.run(J)
        s = DDSolver(c, t, p, eps, dt=dt, precision="fp32_refine", nrhs=nrhs, cg_tol=1e-6)
        probe = tmp_path / f"probe{nrhs}.jsonl"
        s.autotune(probe)
        key = json.loads(probe.read_text().splitlines()[0])["key"]
        f = tmp_path / f"sym{nrhs}.jsonl"
        f.write_text(json.dumps({"key": key, "chunk": 32, "coarse_chunk": 16, "full_chunk": 96,
                                 "full_bucket": 8, "sym_pw": 2, "sym_persist": 16}) + "\n")
        r = s.autotune(f)
        assert r["from_cache"] == 1 and (r["sym_pw"], r["sym_persist"]) == (2, 16)
        assert _err(_steps(s, J), Eo) <= 1e-8, nrhs
