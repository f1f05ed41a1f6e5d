"""The library's host-side partition analysis (Sec. III classes, maps and
orders) built with the address and undefined-behaviour sanitizers by the
host compiler (no device code) and run on regular, uneven, centred and
broken meshes: no sanitizer report, and the counts agree with the HIP
library's own dd_analyze."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from workloads.mesh import centred_cube_mesh, cube_mesh
from workloads.partition import box_partition, rcb_partition

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2204_13254_amd", "csrc")

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("san") / "plan_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
           os.path.join(CSRC, "plan.cpp"), os.path.join(ROOT, "tests", "csrc", "plan_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(driver, tmp_path, c, t, p, name):
    f = tmp_path / f"{name}.bin"
    with open(f, "wb") as fh:
        fh.write(np.array([len(c), len(t)], dtype=np.int64).tobytes())
        fh.write(np.ascontiguousarray(c, dtype=np.float64).tobytes())
        fh.write(np.ascontiguousarray(t, dtype=np.int32).tobytes())
        fh.write(np.ascontiguousarray(p, dtype=np.int32).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([driver, str(f)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
    return r.stdout.split()


def _cases():
    c, t, _ = cube_mesh(6)
    yield "box", c, t, box_partition(6, (2, 3, 1))
    c, t, _ = cube_mesh(8, 1.5)
    yield "rcb_graded", c, t, rcb_partition(8, 4, 3)
    c, t, _ = centred_cube_mesh(4)
    yield "centred", c, t, np.repeat(box_partition(4, 2)[::6], 12)
    c, t, _ = cube_mesh(5)
    yield "one_subdomain", c, t, np.zeros(len(t), dtype=np.int32)


@pytest.mark.parametrize("k", range(4))
def test_analysis_clean_under_sanitizers(driver, tmp_path, k):
    from paper_2204_13254_amd.solver import analyze
    name, c, t, p = list(_cases())[k]
    out = _run(driver, tmp_path, c, t, p, name)
    assert out[:2] == ["rc", "0"], out
    v = dict(zip(out[2::2], (int(x) for x in out[3::2])))
    a, _ = analyze(c, t, p)
    assert (v["ne"], v["nint"], v["nsub"], v["nlam"], v["ncorner"], v["maxmult"]) == \
        (a.n_edges, a.n_interior, a.n_sub, a.n_lambda, a.n_corner, a.max_multiplicity)
    assert v["faces"] == 0 and v["boundary"] > 0


def test_bad_meshes_clean_under_sanitizers(driver, tmp_path):
    c, t, _ = cube_mesh(3)
    p = box_partition(3, 2)
    bad = t.copy(); bad[2, 3] = len(c) + 9                 # vertex out of range
    assert _run(driver, tmp_path, c, bad, p, "range")[:2] == ["rc", "-2"]
    bad = t.copy(); bad[5, 1] = bad[5, 2]                  # repeated vertex
    assert _run(driver, tmp_path, c, bad, p, "degenerate")[:2] == ["rc", "-2"]
    assert _run(driver, tmp_path, c, t, p + 1, "empty")[:2] == ["rc", "-3"]
    q = p.copy(); q[0] = -1
    assert _run(driver, tmp_path, c, t, q, "negative")[:2] == ["rc", "-3"]
