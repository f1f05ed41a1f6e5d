"""CPU tests of the library's host-side partition analysis (Sec. III classes
of unknowns and the Boolean interface maps) and of the C ABI surface.  No
device calls: dd_analyze runs entirely on the host."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.fem import Discretisation
from workloads.configs import workload
from workloads.mesh import cube_mesh
from workloads.partition import box_partition, rcb_partition

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2204_13254_amd._lib import load
    return load()


def test_all_declared_symbols_exported(lib):
    hdr = open(os.path.join(ROOT, "include", "ddfem.h")).read()
    names = set(re.findall(r"\b(dd_[a-z_]+)\s*\(", hdr))
    assert len(names) >= 15
    so = ctypes.CDLL(os.path.join(ROOT, "paper_2204_13254_amd", "libddfem.so"))
    for n in sorted(names):
        assert hasattr(so, n), n


def _analysis(c, t, p):
    from paper_2204_13254_amd.solver import analyze
    return analyze(c, t, p)


@pytest.mark.parametrize("k,expect", [
    (1, (4184, 3032, 8, 480, 24)),
    (2, (102024, 91656, 64, 13824, 648)),
])
def test_counts_of_workloads(k, expect):
    w = workload(k)
    c, t = w.mesh()
    a, per = _analysis(c, t, w.partition())
    assert (a.n_edges, a.n_interior, a.n_sub, a.n_lambda, a.n_corner) == expect
    assert a.max_multiplicity == 4


def _brute_classes(c, t, p):
    """Multiplicity of every interior edge by brute force over tetrahedra,
    using the oracle's own edge numbering."""
    d = Discretisation(c, t)
    subs_of = [set() for _ in range(d.n_e)]
    for tt in range(len(t)):
        for e in d.tet_edges[tt]:
            subs_of[e].add(int(p[tt]))
    return d, subs_of


@pytest.mark.parametrize("n,parts", [(4, 2), (6, ("rcb", 3, 4)), (5, (1, 2, 3))])
def test_classes_and_lambda_map_brute_force(n, parts):
    from paper_2204_13254_amd.solver import analyze_lambda
    c, t, _ = cube_mesh(n)
    p = rcb_partition(n, parts[1], parts[2]) if isinstance(parts, tuple) and parts[0] == "rcb" \
        else box_partition(n, parts)
    a, per = _analysis(c, t, p)
    d, subs_of = _brute_classes(c, t, p)
    inter = [e for e in range(d.n_e) if not d.pec[e]]
    nI = np.zeros(a.n_sub, int); nG = np.zeros(a.n_sub, int); nC = np.zeros(a.n_sub, int)
    gam = []
    for e in inter:
        m = len(subs_of[e])
        for s in subs_of[e]:
            (nI if m == 1 else nG if m == 2 else nC)[s] += 1
        if m == 2:
            gam.append(e)
    assert np.array_equal(per[:, 0], nI) and np.array_equal(per[:, 1], nG) and np.array_equal(per[:, 2], nC)
    assert a.n_lambda == len(gam)
    L = analyze_lambda(c, t, p, a.n_lambda)
    assert np.array_equal(L["edge"], np.array(gam))          # ascending canonical edge id
    for l, e in enumerate(gam):
        lo, hi = sorted(subs_of[e])
        assert (L["sub_lo"][l], L["sub_hi"][l]) == (lo, hi)
    # positions: interface rows come after the interior rows of each subdomain
    assert np.all(L["pos_lo"] >= per[L["sub_lo"], 0])
    assert np.all(L["pos_lo"] < per[L["sub_lo"], 0] + per[L["sub_lo"], 1])
    # B_s jump of a continuous field vanishes: each multiplier sees the same
    # edge from both sides (+1 lo, -1 hi), so sum_s B_s R_s e = e - e = 0
    x = np.random.default_rng(0).standard_normal(d.n_e)
    assert np.allclose(x[L["edge"]] - x[L["edge"]], 0.0)


def test_rejects_bad_inputs(lib):
    from paper_2204_13254_amd._lib import DDError
    c, t, _ = cube_mesh(2)
    p = box_partition(2, 2)
    bad = t.copy(); bad[3, 1] = bad[3, 0]
    with pytest.raises(DDError, match="DD_ERR_MESH"):
        _analysis(c, bad, p)
    bad = t.copy(); bad[0, 0] = len(c) + 5
    with pytest.raises(DDError, match="DD_ERR_MESH"):
        _analysis(c, bad, p)
    with pytest.raises(DDError, match="DD_ERR_PARTITION"):
        _analysis(c, t, p + 1)       # subdomain 0 empty
    flat = c.copy(); flat[:, 2] = 0.0
    with pytest.raises(DDError, match="DD_ERR_MESH"):
        _analysis(flat, t, p)
