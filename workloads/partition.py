"""Seeded partitions of the structured cube mesh into non-overlapping
subdomains (the decomposition of the domain into N_v volumes, Sec. III).

The paper splits its meshes with METIS; those meshes are not available, so
these generators produce box partitions and an index-space recursive
bisection that gives uneven subdomains.  Both assign whole hexahedra (all six
tetrahedra of a hexahedron) to one subdomain.  Output: one int32 subdomain id
per tetrahedron, in tetrahedron id order.
"""
from __future__ import annotations

import numpy as np

from .mesh import hex_ijk


def box_cuts(n: int, parts: int):
    """Hexahedron-aligned cut positions round(linspace(0, n, parts + 1))."""
    return np.round(np.linspace(0, n, parts + 1)).astype(np.int64)


def box_partition(n: int, parts):
    """Split the n^3 hexahedra into parts[0] x parts[1] x parts[2] boxes.

    Box (bi, bj, bk) gets id (bi*parts[1] + bj)*parts[2] + bk.
    """
    if np.isscalar(parts):
        parts = (int(parts),) * 3
    hi, hj, hk = hex_ijk(n)
    ids = []
    for ax, h in enumerate((hi, hj, hk)):
        cuts = box_cuts(n, parts[ax])
        ids.append(np.searchsorted(cuts, h, side="right") - 1)
    box = (ids[0] * parts[1] + ids[1]) * parts[2] + ids[2]
    return np.repeat(box.astype(np.int32), 6)


def rcb_partition(n: int, levels: int, seed: int, frac=(0.4, 0.6)):
    """Index-space recursive bisection with seeded random cut positions.

    Boxes are processed breadth first, left to right.  At each box the axis
    is drawn with rng.choice among the axes of largest hexahedron extent,
    then f ~ U[frac]; the cut sits at lo + round(f*extent), clamped to
    [lo+1, hi-1].  The 2**levels leaves are numbered in breadth-first order.
    """
    rng = np.random.default_rng(seed)
    boxes = [((0, 0, 0), (n, n, n))]
    for _ in range(levels):
        nxt = []
        for lo, hi in boxes:
            ext = [hi[a] - lo[a] for a in range(3)]
            m = max(ext)
            if m < 2:
                raise ValueError("box too small to bisect")
            cand = [a for a in range(3) if ext[a] == m]
            ax = int(rng.choice(cand))
            f = rng.uniform(frac[0], frac[1])
            cut = lo[ax] + int(round(f * ext[ax]))
            cut = min(max(cut, lo[ax] + 1), hi[ax] - 1)
            hi_l = list(hi); hi_l[ax] = cut
            lo_r = list(lo); lo_r[ax] = cut
            nxt.append((lo, tuple(hi_l)))
            nxt.append((tuple(lo_r), hi))
        boxes = nxt
    hi_, hj_, hk_ = hex_ijk(n)
    part = np.full(n ** 3, -1, dtype=np.int64)
    for b, (lo, hi) in enumerate(boxes):
        m = ((hi_ >= lo[0]) & (hi_ < hi[0]) & (hj_ >= lo[1]) & (hj_ < hi[1])
             & (hk_ >= lo[2]) & (hk_ < hi[2]))
        part[m] = b
    assert (part >= 0).all()
    return np.repeat(part.astype(np.int32), 6)
