"""GPU parity of gh_cont (continuation, the paper's surface-following
comparator) with the oracle, through the C ABI: the cells reached and the
distinct lattice points evaluated are identical, marching cubes on them give
the twin's mesh, and with one seed per surface component the cells reached
are exactly the sign-change cells of enumeration."""
import numpy as np
import pytest
from scipy import ndimage

import workloads as W
from oracle import cont as ocont
from oracle import hop as ohop
from oracle import mc as omc
from oracle import sdb as osdb

from test_gpu_prims import _canon, _check_against_twin

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05778_amd import native, polygonize
    return native, polygonize


def component_seeds(cells, n):
    """One cell id per face-connected component of the given cells."""
    grid = np.zeros(n ** 3, dtype=bool)
    grid[cells] = True
    lab, k = ndimage.label(grid.reshape(n, n, n))
    flat = lab.reshape(-1)
    firsts = [int(np.flatnonzero(flat == c)[0]) for c in range(1, k + 1)]
    return np.array(firsts, dtype=np.int64)


def _run_cont(gh, recs, n, lo, h, seeds):
    import torch
    native, P = gh
    poly = P.Polygonizer(P.Bound.prims(recs), n, lo, h)
    m = poly.run(seeds=torch.tensor(seeds, dtype=torch.int64, device="cuda"))
    out = {
        "cand": poly.candidates().cpu().numpy(), "ctr": m.counters,
        "verts": m.verts.cpu().numpy().astype(np.float64),
        "edge": m.vert_edge.cpu().numpy(), "t": m.vert_t.cpu().numpy().astype(np.float64),
        "tris": m.tris.cpu().numpy().astype(np.int64),
        "cells": m.cells.cpu().numpy(), "cases": m.cases.cpu().numpy(),
    }
    out["tri_e"] = _canon(out["edge"][out["tris"]]) if len(out["tris"]) else np.zeros((0, 3), np.int64)
    return out


@pytest.mark.parametrize("scene,n", [("sphere", 64), ("csg0", 96), ("csg2", 57), ("prims0", 80), ("twospheres", 40),
                                     ("sierpinski4", 64)])
def test_cont_matches_oracle(gh, scene, n):
    recs = {"sphere": W.sphere_scene(), "prims0": W.primitives_scene(0), "sierpinski4": W.sierpinski_scene(4),
            "twospheres": np.concatenate([W.sphere_scene(0.3, (-0.45, 0.0, 0.0)),
                                          W.sphere_scene(0.25, (0.5, 0.1, 0.0))])}.get(scene)
    if recs is None:
        recs = W.csg_scene(int(scene[3:]))
    n, lo, h = W.grid(n)
    S = osdb.SDB.prims(recs)
    dense, _ = omc.enumerate_mesh(S, n, lo, h, precision="f32")
    seeds = component_seeds(dense.cells, n)
    out = _run_cont(gh, recs, n, lo, h, seeds)
    cells, evals = ocont.cont(S, n, lo, h, seeds, "f32")
    print(f"{scene} n={n}: components {len(seeds)}, cells {len(cells)}, evals {evals}", flush=True)
    if scene.startswith("sierpinski"):
        # tetrahedra smaller than a cell leave face-adjacent sign-change
        # cells without a sign change on their shared face, so one seed per
        # face-adjacent cluster reaches only part of them
        assert 0 < len(cells) < len(dense.cells)
    else:
        np.testing.assert_array_equal(cells, dense.cells)
    ref = ohop.polygonize_cells(S, n, float(lo), float(h), cells, evals, None, "f32")
    _check_against_twin(out, ref, float(n), float(lo), float(h))


def test_one_seed_reaches_its_component_only(gh):
    recs = np.concatenate([W.sphere_scene(0.3, (-0.45, 0.0, 0.0)), W.sphere_scene(0.25, (0.5, 0.1, 0.0))])
    n, lo, h = W.grid(40)
    S = osdb.SDB.prims(recs)
    dense, _ = omc.enumerate_mesh(S, n, lo, h, precision="f32")
    left = dense.cells[dense.cells // (n * n) < n // 2]
    # seeds outside the grid are ignored; a repeated seed counts once
    out = _run_cont(gh, recs, n, lo, h, np.array([left[3], -5, n ** 3, left[3]], dtype=np.int64))
    np.testing.assert_array_equal(out["cand"], left)
    cells, evals = ocont.cont(S, n, lo, h, [left[3]], "f32")
    assert out["ctr"]["n_hop_evals"] == evals


def test_frontier_capacity_is_flagged(gh):
    import torch
    native, P = gh
    n, lo, h = W.grid(64)
    S = osdb.SDB.prims(W.sphere_scene())
    dense, _ = omc.enumerate_mesh(S, n, lo, h, precision="f32")
    poly = P.Polygonizer(P.Bound.prims(W.sphere_scene()), n, lo, h)
    seeds = torch.tensor(dense.cells[:1], dtype=torch.int64, device="cuda")
    poly.enqueue_cont(seeds, frontier_cap=4)
    c = P.counters_dict(poly.ctr)
    assert c["flags"] & native.GH_FLAG_CAPACITY
    with pytest.raises(native.GhError):           # more seeds than the frontier holds
        poly.enqueue_cont(torch.tensor(dense.cells[:8], dtype=torch.int64, device="cuda"), frontier_cap=4)


def test_full_size_cont_n512(gh):
    # one seed per component of the grid-hopping mesh's cells: continuation
    # reaches exactly those cells, evaluating each of their corners once
    import torch
    native, P = gh
    n, lo, h = W.grid(512)
    recs = W.csg_scene(0)
    poly = P.Polygonizer(P.Bound.prims(recs), n, lo, h)
    sign_cells = poly.run().cells.cpu().numpy()
    seeds = component_seeds(sign_cells, n)
    levels = poly.enqueue_cont(torch.tensor(seeds, dtype=torch.int64, device="cuda"))
    c = P.counters_dict(poly.ctr)
    got = poly.candidates().cpu().numpy()
    print(f"N=512 csg0: components {len(seeds)}, levels {levels}, cells {len(got)}, evals {c['n_hop_evals']}",
          flush=True)
    assert c["flags"] == 0
    np.testing.assert_array_equal(got, sign_cells)
    assert c["n_hop_evals"] == len(ohop.corner_points(n, got))


def test_no_seeds_and_networks(gh):
    # no seed reaches nothing; a network bound is refused
    import torch
    native, P = gh
    n, lo, h = W.grid(32)
    poly = P.Polygonizer(P.Bound.prims(W.sphere_scene()), n, lo, h)
    levels = poly.enqueue_cont(torch.zeros(0, dtype=torch.int64, device="cuda"))
    c = P.counters_dict(poly.ctr)
    assert levels == 0 and c["n_cand"] == 0 and c["n_hop_evals"] == 0 and c["flags"] == 0
    poly = P.Polygonizer(P.Bound.mlp(W.neural_scene(0, 64), "fp32"), n, lo, h)
    with pytest.raises(native.GhError) as e:
        poly.enqueue_cont(torch.zeros(1, dtype=torch.int64, device="cuda"))
    assert e.value.status == native.GH_EUNSUPPORTED
