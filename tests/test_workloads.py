"""Host checks: the centred cube mesh generator (inputs only) gives a
conforming tetrahedralisation of the unit cube, and bench.py refuses more
than one GPU."""
import numpy as np

from oracle.fem import barycentric_gradients, canonical_edges
from oracle.mixed import canonical_faces
from workloads.mesh import centred_cube_mesh


def test_centred_cube_mesh_is_conforming():
    n = 3
    c, t, h = centred_cube_mesh(n)
    assert len(t) == 12 * n ** 3 and len(c) == (n + 1) ** 3 + n ** 3
    _, vol = barycentric_gradients(c, t)
    assert vol.min() > 0 and abs(vol.sum() - 1.0) <= 1e-12
    edges, _ = canonical_edges(t)
    faces, tf = canonical_faces(t)
    use = np.bincount(tf.ravel())
    assert set(np.unique(use)) == {1, 2}                 # boundary faces once, inner faces twice
    assert (use == 1).sum() == 6 * 2 * n * n             # two triangles per boundary square
    assert len(c) - len(edges) + len(faces) - len(t) == 1


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; asked for more it exits with status 2 and a
    message, before touching any device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
