"""Pins of the oracle's literal Algorithm 1 (sphere tracing to the
polygonization distance, Section 3) against closed forms for the two plane
cases the paper analyses (Section 4.1): a plane parallel to the rays and a
plane perpendicular to them.  Both precisions of the oracle must meet them.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import sdb as osdb
from oracle import traced


N, LO, H = 16, -1.0, 0.125          # h = 2/N: every centroid exact in both precisions
TAU = math.sqrt(6.0) / 2.0 * H      # eq. polydist


def _z(k):
    return LO + (k + 0.5) * H


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_plane_parallel_to_rays(precision):
    # f = x - C is constant along every ray.  A column with |x_i - C| <= tau
    # stops its trace at once in every cell: all N cells are candidates and
    # the column takes N + 1 evaluations (the last one at cell N, which is
    # past the top).  Any other column never gets near: its single trace
    # advances by |x_i - C| per evaluation until the travel reaches
    # 1.05 (z_top - z_0), i.e. ceil(1.05 (N - 1/2) h / |x_i - C|)
    # evaluations, and ends beyond the overrun height with no candidate.
    C = 0.1234
    S = osdb.SDB.prims(W.plane_scene((1.0, 0.0, 0.0), C))
    cells, total, per_col = traced.hop_traced(S, N, LO, H, precision)
    tmax = 1.05 * (N - 0.5) * H
    exp_cells, exp_total = [], 0
    for i in range(N):
        dx = abs(_z(i) - C)
        if dx <= TAU:
            exp_total += N * (N + 1)
            exp_cells += [(i * N + j) * N + k for j in range(N) for k in range(N)]
        else:
            r = tmax / dx
            assert abs(r - round(r)) > 1e-3  # no tie: the closed form is unambiguous
            exp_total += N * math.ceil(r)
    assert sum(1 for i in range(N) if abs(_z(i) - C) <= TAU) == 2
    assert total == exp_total
    np.testing.assert_array_equal(cells, np.array(sorted(exp_cells), dtype=np.int64))
    assert per_col.sum() == total


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_plane_perpendicular_to_rays(precision):
    # f = z - C with C = 0.3 (between centroids z_9 = 0.1875 and z_10 = 0.3125).
    # Worked by hand for every column alike:
    #   cell 0: d = 1.2375 > tau, one step of the trace lands on the plane,
    #           d = 0 stops it; the last centroid at or below z = 0.3 is
    #           cell 9: candidate (2 evaluations)
    #   cell 10: d = 0.0125 <= tau: candidate (1)
    #   cell 11: d = 0.1375 <= tau = 0.1531: candidate (1)
    #   cell 12: d = 0.2625 > tau, t = 0.2625 < 1.05 (1 - 0.5625) = 0.4594;
    #           d = 0.525 at z = 0.825, t = 0.7875 >= 0.4594: the trace ends
    #           at z = 1.35, past the overrun height 1.05: the column ends (2)
    C = 0.3
    S = osdb.SDB.prims(W.plane_scene((0.0, 0.0, 1.0), C))
    cells, total, per_col = traced.hop_traced(S, N, LO, H, precision)
    assert _z(11) - C <= TAU < _z(12) - C
    assert total == 6 * N * N
    assert np.all(per_col == 6)
    exp = sorted((c * N) + k for c in range(N * N) for k in (9, 10, 11))
    np.testing.assert_array_equal(cells, np.array(exp, dtype=np.int64))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_plane_near_the_top_uses_the_overrun(precision):
    # f = z - 0.6, worked by hand for every column alike:
    #   cell 0: d = 1.5375, one trace step lands on the plane: cell 12 (2)
    #   cell 13: d = 0.0875 <= tau: candidate (1)
    #   cell 14: d = 0.2125 > tau, t = 0.2125 >= 1.05 (1 - 0.8125) = 0.1969:
    #           the trace ends at z = 1.025, above the top face z = 1 but
    #           not above the overrun height 1.05, and the last centroid at or
    #           below it is cell 15: candidate (1)
    #   cell 16 (past the top): d = 0.4625, the travel limit is negative, the
    #           trace ends at z = 1.525: the column ends (1)
    C = 0.6
    S = osdb.SDB.prims(W.plane_scene((0.0, 0.0, 1.0), C))
    cells, total, per_col = traced.hop_traced(S, N, LO, H, precision)
    assert np.all(per_col == 5) and total == 5 * N * N
    exp = sorted((c * N) + k for c in range(N * N) for k in (12, 13, 15))
    np.testing.assert_array_equal(cells, np.array(exp, dtype=np.int64))


def test_precisions_agree_on_sphere_up_to_rounding():
    # Same procedure in both precisions on a sphere at N = 32: the candidate
    # sets may differ only where float32 rounding moves a trace across tau or
    # a cell boundary, which is rare.
    n, lo, h = W.grid(32)
    S = osdb.SDB.prims(W.sphere_scene())
    c64, e64, _ = traced.hop_traced(S, n, lo, h, "f64")
    c32, e32, _ = traced.hop_traced(S, n, lo, h, "f32")
    diff = len(np.setxor1d(c64, c32))
    assert diff <= max(1, len(c64) // 1000), diff
    assert abs(e64 - e32) <= max(1, e64 // 1000)
