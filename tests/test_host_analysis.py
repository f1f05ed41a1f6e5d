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


# (n_e, N_int, subdomains, n_lambda, n_c) and the min-max of n_r = n_I + n_Gamma
# per subdomain, as tabulated for the five workloads in the design survey
# (computed there by independent scripts)
@pytest.mark.parametrize("k,expect,nr_range", [
    (1, (4184, 3032, 8, 480, 24), (436, 436)),
    (2, (102024, 91656, 64, 13824, 648), (1494, 1782)),
    pytest.param(3, (795024, 753552, 512, 124115, 11934), (394, 4474), marks=pytest.mark.slow),
    pytest.param(4, (238688, 220256, 64, 25344, 864), (3560, 4088), marks=pytest.mark.slow),
    pytest.param(5, (1872064, 1798336, 1000, 297216, 15552), (1494, 2779), marks=pytest.mark.slow),
])
def test_counts_of_workloads(k, expect, nr_range):
    w = workload(k)
    c, t = w.mesh()
    a, per = _analysis(c, t, w.partition())
    assert (a.n_edges, a.n_interior, a.n_sub, a.n_lambda, a.n_corner) == expect
    assert a.max_multiplicity == 4
    nr = per[:, 0] + per[:, 1]
    assert (int(nr.min()), int(nr.max())) == nr_range


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
    # positions: the interface block of a subdomain follows its interior
    # block, and every interface edge of the subdomain is one multiplier's
    # side there: the positions of the multipliers that enter a subdomain
    # cover its interface block exactly once, and the edges found there are
    # the brute-force interface edges of that subdomain (in the library's
    # own order of the block)
    gam_of = [[-1] * int(per[s, 1]) for s in range(a.n_sub)]
    for side in ("lo", "hi"):
        sub, pos = L["sub_" + side], L["pos_" + side]
        off = pos - per[sub, 0]
        assert np.all(off >= 0) and np.all(off < per[sub, 1])
        for s_, o, e in zip(sub, off, L["edge"]):
            assert gam_of[s_][o] == -1
            gam_of[s_][o] = int(e)
    for s in range(a.n_sub):
        assert sorted(gam_of[s]) == sorted(e for e in gam if s in subs_of[e])

    # restriction R_s of an edge field to each subdomain's interface rows
    def restrict(x):
        return [x[np.array(g, dtype=np.int64)] if g else np.zeros(0) for g in gam_of]

    def jump(xs):    # sum_s B_s x_s: +1 in the lower subdomain id, -1 in the higher
        lo = np.array([xs[s_][o] for s_, o in zip(L["sub_lo"], L["pos_lo"] - per[L["sub_lo"], 0])])
        hi = np.array([xs[s_][o] for s_, o in zip(L["sub_hi"], L["pos_hi"] - per[L["sub_hi"], 0])])
        return lo - hi

    # a continuous field has no jump; a field torn in one subdomain jumps by
    # exactly the tear on that subdomain's multipliers, with its sign
    x = np.random.default_rng(0).integers(-1000, 1000, d.n_e).astype(np.float64)   # exact sums
    assert np.array_equal(jump(restrict(x)), np.zeros(a.n_lambda))
    xs = restrict(x)
    s_t = int(L["sub_hi"][0])
    xs[s_t] = xs[s_t] + 1.0
    j = jump(xs)
    np.testing.assert_array_equal(j, np.where(L["sub_hi"] == s_t, -1.0, 0.0)
                                  + np.where(L["sub_lo"] == s_t, 1.0, 0.0))


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
