"""Pins of the oracle's continuation (the paper's surface-following
comparator, Section 2): on a connected surface, one seed reaches exactly the
sign-change cells of enumeration (a separate code path), and it evaluates
exactly the distinct corners of those cells."""
import numpy as np
import pytest

import workloads as W
from oracle import cont as ocont
from oracle import hop as ohop
from oracle import mc as omc
from oracle import sdb as osdb


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_sphere_one_seed_reaches_every_sign_change_cell(precision):
    n, lo, h = W.grid(32)
    S = osdb.SDB.prims(W.sphere_scene())
    dense, _ = omc.enumerate_mesh(S, n, lo, h, precision=precision)
    seed = dense.cells[len(dense.cells) // 2]
    cells, evals = ocont.cont(S, n, lo, h, [seed], precision)
    np.testing.assert_array_equal(cells, dense.cells)
    assert evals == len(ohop.corner_points(n, cells))


def test_one_seed_per_component():
    # two disjoint spheres: a seed in one reaches that sphere only; a seed in
    # each reaches both, i.e. all of enumeration's sign-change cells
    n, lo, h = W.grid(40)
    recs = np.concatenate([W.sphere_scene(0.3, (-0.45, 0.0, 0.0)), W.sphere_scene(0.25, (0.5, 0.1, 0.0))])
    S = osdb.SDB.prims(recs)
    dense, _ = omc.enumerate_mesh(S, n, lo, h, precision="f32")
    i = dense.cells // (n * n)
    left, right = dense.cells[i < n // 2], dense.cells[i >= n // 2]
    one, _ = ocont.cont(S, n, lo, h, [left[0]], "f32")
    np.testing.assert_array_equal(one, left)
    both, _ = ocont.cont(S, n, lo, h, [left[0], right[-1]], "f32")
    np.testing.assert_array_equal(both, dense.cells)


def test_seed_off_the_surface_reaches_only_itself():
    n, lo, h = W.grid(16)
    S = osdb.SDB.prims(W.sphere_scene())
    cells, evals = ocont.cont(S, n, lo, h, [0], "f32")    # a corner cell, far outside
    np.testing.assert_array_equal(cells, [0])
    assert evals == 8
