"""The bench's roofline arithmetic on synthetic class timings (host only).

The symmetric product y = M u (M symmetric n_G x n_G per subdomain) moves
n_G(n_G+1)/2 stored entries plus one read of u and one write of y, and costs
2 n_G^2 flops per RHS; the reported bound is the resource with the larger
minimum time (HBM at 8 TB/s, FP32 MFMA at 157.3 TFLOP/s).
"""
import numpy as np

import bench


class _Info:
    def __init__(self, nG):
        self.precision = 1  # FP32 factors
        self.trailing_bytes = self.full_bytes = self.corner_bytes = 1
        self.coarse_bytes = self.cross_bytes = 1
        self.n_corner = 1
        self.schur_bytes = int((nG * (nG + 1) // 2).sum() * 4)


class _Solver:
    def __init__(self, nG):
        self.info = _Info(nG)


def _roof(nG, nrhs, ms):
    per = np.stack([np.zeros_like(nG), nG, np.zeros_like(nG)], 1)
    prof = {k: (1e-6, 1) for k in ("trailing", "full", "corner", "coarse", "cross")}
    prof["schur"] = (4 * ms, 4)
    roof, _ = bench.roofline(_Solver(nG), per, nrhs, prof)
    return roof


def test_hbm_bound_at_16_rhs():
    nG = np.full(100, 600, dtype=np.int64)
    roof = _roof(nG, 16, 0.02)
    bytes_ = (600 * 601 // 2) * 4 * 100 + 2 * 600 * 100 * 16 * 4
    flops = 2 * 16 * 600 * 600 * 100
    assert roof["class"] == "schur" and roof["bound"] == "hbm"
    assert roof["bytes_per_launch"] == bytes_
    assert roof["flops_per_launch"] == flops
    assert abs(roof["achieved"] - bytes_ / 0.02e-3 / 1e9) < 0.1
    assert abs(roof["mfma_tflops"] - flops / 0.02e-3 / 1e12) < 0.01
    # MFMA time over HBM time, both at their peaks
    ratio = (flops / 157.3e12) / (bytes_ / 8e12)
    assert abs(roof["mfma_over_hbm_time"] - round(ratio, 3)) < 1e-3 and ratio < 1


def test_mfma_bound_at_32_rhs():
    nG = np.full(100, 600, dtype=np.int64)
    roof = _roof(nG, 32, 0.03)
    flops = 2 * 32 * 600 * 600 * 100
    bytes_ = (600 * 601 // 2) * 4 * 100 + 2 * 600 * 100 * 32 * 4
    assert roof["bound"] == "mfma" and roof["unit"] == "TFLOP/s" and roof["peak"] == 157.3
    assert abs(roof["achieved"] - flops / 0.03e-3 / 1e12) < 0.01
    assert abs(roof["frac"] - roof["achieved"] / 157.3) < 1e-4
    # the HBM figures stay beside it
    assert abs(roof["hbm_achieved_GBps"] - bytes_ / 0.03e-3 / 1e9) < 0.1
    assert abs(roof["hbm_frac"] - roof["hbm_achieved_GBps"] / 8000.0) < 1e-4


def test_committed_counter_summary_matches_the_kernel_sources():
    # the committed FETCH/WRITE summary of every product class was taken on
    # the current kernel sources of the 64^3 workload (else the bench reports
    # no traffic); another workload never borrows it
    for cls in ("full", "cross", "schur"):
        v = bench._profiled_class(cls, "cavity64_box10_beam16")
        assert v is not None, cls
        assert v["bytes_per_launch"] > 0 and v["rocprof_avg_ms"] > 0
        assert bench._profiled_class(cls, "graded48_rcb512_32rhs") is None
