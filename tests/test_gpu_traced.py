"""GPU parity of gh_hop_traced (the paper's per-column procedure taken
literally) with the oracle's FP32 twin of it, through the C ABI: candidate
cells and evaluation counts are identical, and marching cubes on them give
the twin's mesh.  The missed-cell audit (sign-change cells the rule leaves
out) is printed and must agree with the oracle's."""
import numpy as np
import pytest

import workloads as W
from oracle import sdb as osdb
from oracle import traced as otr

from test_gpu_prims import _check_against_twin, _canon

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05778_amd import native, polygonize
    return native, polygonize


def _run_traced(gh, recs, n, lo, h, lanes=0):
    native, P = gh
    poly = P.Polygonizer(P.Bound.prims(recs), n, lo, h)
    native.gh_set_tuning(hop_lanes_per_ray=lanes)
    try:
        m = poly.run(traced=True)
    finally:
        native.gh_set_tuning(0)
    cand = poly.candidates().cpu().numpy()
    out = {
        "cand": cand, "ctr": m.counters,
        "verts": m.verts.cpu().numpy().astype(np.float64),
        "edge": m.vert_edge.cpu().numpy(), "t": m.vert_t.cpu().numpy().astype(np.float64),
        "tris": m.tris.cpu().numpy().astype(np.int64),
        "cells": m.cells.cpu().numpy(), "cases": m.cases.cpu().numpy(),
    }
    out["tri_e"] = _canon(out["edge"][out["tris"]]) if len(out["tris"]) else np.zeros((0, 3), np.int64)
    return out


def _scene(name):
    if name == "sphere":
        return W.sphere_scene()
    if name == "xplane":
        return W.plane_scene((1.0, 0.0, 0.0), 0.1234)
    if name == "zplane_top":
        return W.plane_scene((0.0, 0.0, 1.0), 0.6)
    if name == "box":
        return W.box_scene((0.31, 0.2, 0.45), (0.05, -0.1, 0.02))
    if name == "genus2":
        return W.genus2_scene()
    if name.startswith("prims"):
        return W.primitives_scene(int(name[5:]))
    if name.startswith("sierpinski"):
        return W.sierpinski_scene(int(name[10:]))
    return W.csg_scene(int(name[3:]))


@pytest.mark.parametrize("scene,n,lanes", [
    ("sphere", 64, 0), ("csg0", 64, 0), ("csg1", 100, 0), ("csg2", 37, 0), ("csg3", 128, 1), ("csg4", 48, 8),
    ("box", 50, 0), ("xplane", 16, 0), ("zplane_top", 16, 0), ("csg0", 1, 0), ("csg0", 2, 0), ("csg7", 61, 4),
    ("prims0", 80, 0), ("genus2", 32, 0), ("sierpinski5", 72, 0), ("sierpinski3", 40, 2)])
def test_traced_matches_fp32_twin(gh, scene, n, lanes):
    recs = _scene(scene)
    g = W.grid(n)
    out = _run_traced(gh, recs, *g, lanes=lanes)
    ref = otr.gridhop_traced(osdb.SDB.prims(recs), *g, precision="f32")
    print(f"{scene} n={n}: evals={ref.hop_evals} cand={len(ref.candidates)} cells={len(ref.mesh.cells)}", flush=True)
    _check_against_twin(out, ref, *[float(x) for x in g])


@pytest.mark.parametrize("scene", ["csg0", "csg1", "sphere"])
def test_traced_full_size_counts_and_audit(gh, scene):
    # N = 512: candidate cells and evaluation counts equal the twin's; the
    # audit of sign-change cells (those of the grid-hopping mesh, which is
    # the enumeration's) that the literal rule leaves out is the twin's too
    import torch
    native, P = gh
    recs = _scene(scene)
    n, lo, h = W.grid(512)
    cells, total, _ = otr.hop_traced(osdb.SDB.prims(recs), n, lo, h, "f32")
    poly = P.Polygonizer(P.Bound.prims(recs), n, lo, h, keep_cells=True)
    m = poly.run()                                   # grid hopping: every sign-change cell
    sign_cells = m.cells.cpu().numpy()
    poly.enqueue_hop_traced()
    torch.cuda.synchronize()
    c = P.counters_dict(poly.ctr)
    assert c["flags"] == 0
    assert c["n_hop_evals"] == total and c["n_cand"] == len(cells)
    got = poly.candidates().cpu().numpy()
    np.testing.assert_array_equal(got, cells)
    missed = np.setdiff1d(sign_cells, got)
    print(f"{scene} N=512: traced evals {total}, candidates {len(cells)}; sign-change cells {len(sign_cells)}, "
          f"missed by the literal rule {len(missed)}", flush=True)
    assert len(missed) == len(np.setdiff1d(sign_cells, cells))


def test_traced_rejects_networks(gh):
    native, P = gh
    b = P.Bound.mlp(W.neural_scene(0, 64), "fp32")
    poly = P.Polygonizer(b, *W.grid(16))
    with pytest.raises(native.GhError) as e:
        poly.enqueue_hop_traced()
    assert e.value.status == native.GH_EUNSUPPORTED
