"""GPU parity of the analytic path against the oracle, through the C ABI.

Against the oracle's float32 twin (same formula, same op order) the results
must be identical: candidate cells, evaluation counts, distinct corners,
sign-change cells and case bytes, welded vertex edge ids and triangles; the
edge parameters t agree to 1e-5 and positions to 1e-5 h (t is float32 on the
GPU, float64 from the same float32 values in the oracle).  Against the FP64
oracle the sign-change cells agree once cells with a corner |f| below
max(1e-6 h, 2^-20) are set aside; their number is reported.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import hop as ohop
from oracle import mc as omc
from oracle import sdb as osdb

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05778_amd import native, polygonize
    return native, polygonize


def _canon(tri_e):
    if len(tri_e) == 0:
        return tri_e.reshape(0, 3)
    r = np.argmin(tri_e, axis=1)
    t = np.take_along_axis(tri_e, (r[:, None] + np.arange(3)) % 3, axis=1)
    return t[np.lexsort((t[:, 2], t[:, 1], t[:, 0]))]


def _run(gh, recs, n, lo, h, dense=False):
    native, P = gh
    poly = P.Polygonizer(P.Bound.prims(recs), n, lo, h)
    m = poly.run(dense=dense)
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


def _closed_oriented(tris):
    """Every directed edge once, and its reverse present (numpy, any size)."""
    v = int(tris.max()) + 1 if len(tris) else 1
    d = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    key = d[:, 0] * v + d[:, 1]
    rev = d[:, 1] * v + d[:, 0]
    return len(np.unique(key)) == len(key) and np.isin(rev, key).all()


def _check_against_twin(g, ref, n, lo, h, n_cand_ref=None):
    m = ref.mesh
    assert g["ctr"]["flags"] == 0
    assert g["ctr"]["n_hop_evals"] == ref.hop_evals
    assert g["ctr"]["n_cand"] == len(ref.candidates)
    np.testing.assert_array_equal(g["cand"], ref.candidates)
    assert g["ctr"]["n_corner"] == ref.corner_evals
    np.testing.assert_array_equal(g["cells"], m.cells)
    np.testing.assert_array_equal(g["cases"], m.cases)
    np.testing.assert_array_equal(g["edge"], m.edge_ids)
    if len(m.ts):
        assert np.abs(g["t"] - m.ts).max() <= 1e-5
        pos = omc.edge_positions(n, lo, h, m.edge_ids, m.ts)
        assert np.abs(g["verts"] - pos).max() <= 1e-5 * h
    np.testing.assert_array_equal(g["tri_e"], m.tris)
    assert g["ctr"]["n_tri"] == len(m.tris) and g["ctr"]["n_vert"] == len(m.edge_ids)
    assert g["ctr"]["n_cells"] == len(m.cells)


def _named_scene(scene):
    recs = {"sphere": W.sphere_scene(), "box": W.box_scene((0.31, 0.2, 0.45), (0.05, -0.1, 0.02)),
            "boxbound": W.box_scene((0.31, 0.2, 0.45), (0.05, -0.1, 0.02), bound=True),
            "cylinder": W.cylinder_scene(0.37, 0.29, (0.03, -0.05, 0.01)),
            "cone": W.cone_scene(0.41, 0.45, (-0.02, 0.04, 0.0)),
            "hexprism": W.hexprism_scene(0.33, 0.27, (0.02, 0.01, -0.03)),
            "genus2": W.genus2_scene()}.get(scene)
    if recs is None and scene.startswith("sierpinski"):
        recs = W.sierpinski_scene(int(scene[10:]))
    if recs is None and scene.startswith("prims"):
        recs = W.primitives_scene(int(scene[5:]))
    if recs is None:
        recs = W.csg_scene(int(scene[3:]))
    return recs


@pytest.mark.parametrize("scene,n", [("sphere", 64), ("csg0", 64), ("csg1", 100), ("csg2", 37), ("csg0", 128),
                                     ("box", 50), ("boxbound", 33), ("csg3", 1), ("csg4", 2), ("cylinder", 64),
                                     ("cone", 57), ("hexprism", 64), ("prims0", 128), ("prims1", 75),
                                     ("genus2", 48), ("genus2", 64), ("sierpinski0", 40), ("sierpinski3", 64),
                                     ("sierpinski6", 128), ("sierpinski16", 33)])
def test_matches_fp32_twin(gh, scene, n):
    recs = _named_scene(scene)
    g = W.grid(n)
    out = _run(gh, recs, *g)
    ref = ohop.gridhop(osdb.SDB.prims(recs), *g, precision="f32")
    print(f"{scene} n={n}: evals={ref.hop_evals} cand={len(ref.candidates)} cells={len(ref.mesh.cells)}", flush=True)
    _check_against_twin(out, ref, *[float(x) for x in g])


def _lattice_tile_loads(cells, n, tile=256):
    """Corners and candidates per tile of `tile` consecutive lattice columns
    (a * (n + 1) + b), from a candidate list (numpy)."""
    n1 = n + 1
    col, k = cells // n, cells % n
    i, j = col // n, col % n
    corners = np.unique(np.concatenate([((i + di) * n1 + (j + dj)) * n1 + (k + dk)
                                        for di in (0, 1) for dj in (0, 1) for dk in (0, 1)]))
    per_c = np.bincount(corners // n1 // tile)
    per_k = np.bincount((i * n1 + j) // tile)
    return per_c, per_k


@pytest.mark.parametrize("scene,n", [("plane_x", 128), ("box_walls", 160)])
def test_tiles_beyond_the_stage_match_twin(gh, scene, n):
    """Walls parallel to the lattice columns put far more corners and
    candidates in a tile of 256 lattice columns than the corner pass's LDS
    stage holds (4,096 and 3,072): such a tile writes its lists directly
    after its look-back, with word records relative to the tile's first
    corner.  The mesh still equals the FP32 twin's, and the tile sizes are
    checked on the host so that the path is really taken."""
    if scene == "plane_x":
        recs = W.plane_scene((1, 0, 0), 0.1234)
    else:
        recs = W.box_scene((0.6, 0.55, 0.8), (0.013, -0.021, 0.008))
    g = W.grid(n)
    ref = ohop.gridhop(osdb.SDB.prims(recs), *g, precision="f32")
    per_c, per_k = _lattice_tile_loads(ref.candidates, n)
    print(f"{scene} n={n}: largest tile {per_c.max()} corners, {per_k.max()} candidates", flush=True)
    assert per_c.max() > 4096 and per_k.max() > 3072
    out = _run(gh, recs, *g)
    _check_against_twin(out, ref, *[float(x) for x in g])


def _prim(ptype, centre, params):
    return W._record(ptype, centre, np.eye(3), params)[None, :]


@pytest.mark.parametrize("case", ["zero_radius_at_centroids", "thin_ring", "fine_grid"])
def test_hop_root_conditions(gh, case):
    # The register-record hop takes square roots that are exact from 2^-96 up
    # and clamp below; that gives the exact root's decisions only for cells
    # of at least 2^-20 and torus ring radii of at least 2^-23, and a grid or
    # union outside those takes the kernel with exact roots.  Either way the
    # result is the twin's.
    if case == "fine_grid":
        h = 2.0 ** -22
        n, lo, h = W.grid(48, lo=-24 * h, extent=48 * h)
        recs = np.concatenate([_prim(W.PRIM_SPHERE, (0.0, 0.0, 0.0), (15 * h,)),
                               _prim(W.PRIM_BOX, (5 * h, 3 * h, -4 * h), (9 * h, 6 * h, 11 * h)),
                               _prim(W.PRIM_TORUS, (-6 * h, 2 * h, 1 * h), (12 * h, 3 * h))])
    else:
        n, lo, h = W.grid(40)
        if case == "thin_ring":  # ring radius below 2^-23: a sphere-like torus
            recs = np.concatenate([_prim(W.PRIM_TORUS, (0.1, -0.05, 0.0), (1e-9, 0.45)),
                                   _prim(W.PRIM_CAPSULE, (-0.3, 0.2, 0.1), (0.3, 0.15))])
        else:  # radius-0 spheres and a radius-0 torus tube whose roots see exact zeros at centroids
            c = lambda i, j, k: tuple(float(v) for v in ohop.centroid_f32(lo, h, np.array([i, j, k])))
            recs = np.concatenate([_prim(W.PRIM_SPHERE, c(10, 20, 30), (0.0,)),
                                   _prim(W.PRIM_SPHERE, c(25, 5, 17), (2.0 ** -30,)),
                                   _prim(W.PRIM_TORUS, c(32, 30, 8), (0.25, 0.0)),
                                   _prim(W.PRIM_BOX, (0.1, 0.0, -0.1), (0.3, 0.25, 0.2))])
    out = _run(gh, recs, n, lo, h)
    ref = ohop.gridhop(osdb.SDB.prims(recs), n, lo, h, precision="f32")
    print(f"{case}: evals={ref.hop_evals} cand={len(ref.candidates)} cells={len(ref.mesh.cells)}", flush=True)
    assert ref.hop_evals > n * n
    _check_against_twin(out, ref, float(n), float(lo), float(h))


def test_sphere_n64_against_fp64_oracle(gh):
    n, lo, h = W.grid(64)
    recs = W.sphere_scene()
    out = _run(gh, recs, n, lo, h)
    S = osdb.SDB.prims(recs)
    dense, F = omc.enumerate_mesh(S, n, lo, h)
    thr = max(1e-6 * float(h), 2.0 ** -20)
    near = np.zeros((n, n, n), bool)
    for c in range(8):
        dx, dy, dz = omc.CORNER[c]
        near |= np.abs(F[dx:dx + n, dy:dy + n, dz:dz + n]) < thr
    excl = np.nonzero(near.ravel())[0]
    # the sphere of radius 1/2 passes exactly through lattice points such as
    # (1/2, 0, 0), where f = 0 in both precisions: those cells are set aside
    print(f"excluded cells: {len(excl)}", flush=True)
    assert len(excl) <= 64
    keep_g = out["cells"][~np.isin(out["cells"], excl)]
    keep_o = dense.cells[~np.isin(dense.cells, excl)]
    np.testing.assert_array_equal(keep_g, keep_o)
    # exact zeros are exact in float32 too, so here the full sets agree as well
    np.testing.assert_array_equal(out["cells"], dense.cells)
    np.testing.assert_array_equal(out["tri_e"], dense.tris)
    P = out["verts"]
    T = np.searchsorted(out["edge"], out["tri_e"])
    assert _closed_oriented(T)
    area = 0.5 * np.linalg.norm(np.cross(P[T[:, 1]] - P[T[:, 0]], P[T[:, 2]] - P[T[:, 0]]), axis=1).sum()
    assert abs(area - math.pi) < 5e-3


@pytest.mark.parametrize("scene,n", [("sphere", 48), ("csg0", 64), ("csg1", 77), ("prims0", 96), ("genus2", 40),
                                     ("sierpinski5", 96)])
def test_dense_equals_hop(gh, scene, n):
    recs = _named_scene(scene)
    g = W.grid(n)
    a = _run(gh, recs, *g)
    b = _run(gh, recs, *g, dense=True)
    for key in ("cells", "cases", "edge", "t", "verts", "tri_e"):
        np.testing.assert_array_equal(a[key], b[key])
    assert b["ctr"]["n_hop_evals"] == (n + 1) ** 3
    assert b["ctr"]["n_cand"] == len(b["cells"])
    # the dense classification is the enumeration of the twin
    ref, _ = omc.enumerate_mesh(osdb.SDB.prims(recs), *g, precision="f32")
    np.testing.assert_array_equal(b["cand"], ref.cells)


def test_full_size_csg_n512_matches_twin(gh):
    n, lo, h = W.grid(512)
    recs = W.csg_scene(0)
    out = _run(gh, recs, n, lo, h)
    ref = ohop.gridhop(osdb.SDB.prims(recs), n, lo, h, precision="f32")
    print(f"N=512 csg0: evals={ref.hop_evals} cand={len(ref.candidates)} corners={ref.corner_evals} "
          f"tris={len(ref.mesh.tris)}", flush=True)
    _check_against_twin(out, ref, n, float(lo), float(h))
    T = np.searchsorted(out["edge"], out["tri_e"])
    assert _closed_oriented(T)


@pytest.mark.parametrize("n", [64, 256, 1024])
def test_plane_perpendicular_count(gh, n):
    g = W.grid(n)
    out = _run(gh, W.plane_scene((0, 0, 1), 0.1234), *g)
    assert out["ctr"]["n_hop_evals"] == n * n * (round(math.log2(n)) + 2)
    assert out["ctr"]["n_cand"] == 2 * n * n


def test_plane_parallel_count(gh):
    n, lo, h = W.grid(256)
    out = _run(gh, W.plane_scene((1, 0, 0), 0.1234), n, lo, h)
    xs = float(lo) + (np.arange(n) + 0.5) * float(h)
    s = np.floor(np.abs(xs - 0.1234) / float(h)).astype(int)
    assert out["ctr"]["n_hop_evals"] == n * int(np.where(s == 0, n, np.ceil(n / np.maximum(s, 1))).sum())


def test_eval_points_bit_exact(gh):
    import torch
    native, P = gh
    recs = W.csg_scene(3)
    b = P.Bound.prims(recs)
    pts = np.random.default_rng(0).uniform(-1, 1, (100000, 3)).astype(np.float32)
    f = b.eval(torch.from_numpy(pts).cuda()).cpu().numpy()
    ref = osdb.union_f32(recs, pts[:, 0], pts[:, 1], pts[:, 2])
    np.testing.assert_array_equal(f, ref)


def test_sqrt_correctly_rounded_over_wide_range(gh):
    """The kernels' square root (hardware estimate + rounding test, library
    path for tiny inputs) against numpy's correctly rounded float32 sqrt:
    a sphere of radius 0 at the origin evaluates sqrt((x x + y y) + z z).
    Magnitudes are log-uniform over [2^-63, 2^60] (sums of squares from the
    smallest normal up, so the tiny-input path is covered), signs random,
    plus exact zeros."""
    import torch
    native, P = gh
    recs = W.sphere_scene(0.0)
    b = P.Bound.prims(recs)
    rng = np.random.default_rng(5)
    m = 1 << 22
    mag = np.exp2(rng.uniform(-63, 60, (m, 3)))
    pts = (mag * rng.choice([-1.0, 1.0], (m, 3))).astype(np.float32)
    pts[:1000] = 0.0
    pts[1000:2000, 1:] = 0.0  # one non-zero component: sqrt of a rounded square
    f = b.eval(torch.from_numpy(pts).cuda()).cpu().numpy()
    ref = osdb.union_f32(recs, pts[:, 0], pts[:, 1], pts[:, 2])
    s = (pts[:, 0] * pts[:, 0] + pts[:, 1] * pts[:, 1]) + pts[:, 2] * pts[:, 2]
    assert (s < np.float32(2.0 ** -96)).sum() > 1000  # the tiny-input path ran
    np.testing.assert_array_equal(f, ref)


def test_capacity_overflow_reports_required_sizes(gh):
    import torch
    native, P = gh
    n, lo, h = W.grid(64)
    recs = W.csg_scene(0)
    poly = P.Polygonizer(P.Bound.prims(recs), n, lo, h, corner_cap=100, vert_cap=10, tri_cap=10, cell_cap=10)
    poly.enqueue_hop()
    poly.enqueue_mc()
    torch.cuda.synchronize()
    c = P.counters_dict(poly.ctr)
    ref = ohop.gridhop(osdb.SDB.prims(recs), n, lo, h, precision="f32")
    assert c["flags"] & native.GH_FLAG_CAPACITY
    assert c["n_corner"] == ref.corner_evals
    # with room for the corners, the vertex and triangle counts are reported too
    poly2 = P.Polygonizer(P.Bound.prims(recs), n, lo, h, vert_cap=10, tri_cap=10, cell_cap=10)
    poly2.enqueue_hop()
    poly2.enqueue_mc()
    torch.cuda.synchronize()
    c2 = P.counters_dict(poly2.ctr)
    assert c2["flags"] & native.GH_FLAG_CAPACITY
    assert c2["n_vert"] == len(ref.mesh.edge_ids) and c2["n_tri"] == len(ref.mesh.tris)
    assert c2["n_cells"] == len(ref.mesh.cells)
    m = poly2.run()                         # grows the buffers and succeeds
    assert m.counters["flags"] == 0 and m.counters["n_tri"] == len(ref.mesh.tris)


def test_nonfinite_bound_flagged(gh):
    native, P = gh
    recs = W.sphere_scene(0.5, centre=(1e30, 0.0, 0.0))
    poly = P.Polygonizer(P.Bound.prims(recs), 16, -1.0, 0.125)
    with pytest.raises(FloatingPointError):
        poly.run()


def test_repeat_runs_identical(gh):
    g = W.grid(96)
    recs = W.csg_scene(5)
    a, b = _run(gh, recs, *g), _run(gh, recs, *g)
    for key in ("cells", "cases", "edge", "t", "verts", "tris"):
        np.testing.assert_array_equal(a[key], b[key])


def test_empty_scene(gh):
    # sphere entirely outside the grid: no candidates, no mesh
    out = _run(gh, W.sphere_scene(0.2, centre=(5.0, 5.0, 5.0)), *W.grid(40))
    assert out["ctr"]["n_cand"] == 0 and out["ctr"]["n_tri"] == 0 and out["ctr"]["n_corner"] == 0


@pytest.mark.parametrize("lanes", [0, 1, 2, 3, 4, 8])
def test_every_hop_shape_matches_twin(gh, lanes):
    native, P = gh
    recs = W.csg_scene(1)
    g = W.grid(100)
    native.gh_set_tuning(hop_lanes_per_ray=lanes)
    try:
        out = _run(gh, recs, *g)
    finally:
        native.gh_set_tuning(0)
    ref = ohop.gridhop(osdb.SDB.prims(recs), *g, precision="f32")
    _check_against_twin(out, ref, *[float(x) for x in g])


def test_counters_repeatable_full_size(gh):
    # per-block partial sums are reused by consecutive reductions; repeated
    # runs and every hop shape must give the oracle's exact counts
    native, P = gh
    n, lo, h = W.grid(512)
    recs = W.csg_scene(0)
    cells, total, _ = ohop.hop(osdb.SDB.prims(recs), n, lo, h, precision="f32")
    b = P.Bound.prims(recs)
    import torch
    try:
        for lanes in (0, 1, 2, 3, 4, 8):
            native.gh_set_tuning(lanes)
            poly = P.Polygonizer(b, n, lo, h, keep_cells=False)
            for _ in range(3):
                poly.enqueue_hop()
                torch.cuda.synchronize()
                c = P.counters_dict(poly.ctr)
                assert c["n_hop_evals"] == total and c["n_cand"] == len(cells), (lanes, c)
    finally:
        native.gh_set_tuning(0)


@pytest.mark.parametrize("n_prim,lanes", [(5, 0), (7, 0), (7, 3), (16, 0), (16, 3), (1, 0)])
def test_uneven_type_groups_match_twin(gh, n_prim, lanes):
    # type groups of unequal size (the built-in lane count follows the
    # largest group; R = 3 leaves lanes idle in smaller groups)
    native, P = gh
    recs = W.csg_scene(7, n_prim)
    g = W.grid(61)
    native.gh_set_tuning(hop_lanes_per_ray=lanes)
    try:
        out = _run(gh, recs, *g)
    finally:
        native.gh_set_tuning(0)
    ref = ohop.gridhop(osdb.SDB.prims(recs), *g, precision="f32")
    _check_against_twin(out, ref, *[float(x) for x in g])


@pytest.mark.parametrize("lanes", [0, 1, 3])
def test_sierpinski_in_a_union_matches_twin(gh, lanes):
    # the fractal beside the other types (records read from LDS, one or
    # three lanes per ray, and the default)
    native, P = gh
    recs = np.concatenate([W.csg_scene(0), W.sierpinski_scene(5, scale=2.0, centre=(0.31, -0.27, 0.22))])
    g = W.grid(80)
    native.gh_set_tuning(hop_lanes_per_ray=lanes)
    try:
        out = _run(gh, recs, *g)
    finally:
        native.gh_set_tuning(0)
    ref = ohop.gridhop(osdb.SDB.prims(recs), *g, precision="f32")
    _check_against_twin(out, ref, *[float(x) for x in g])


@pytest.mark.parametrize("budget,lanes,scene,n_prim,n", [
    (1, 0, 1, 12, 100), (4, 3, 1, 12, 100), (16, 1, 1, 12, 100), (2, 8, 1, 12, 100), (0, 0, 1, 12, 100),
    (3, 0, 7, 24, 61), (1, 4, 7, 5, 61), (2, 0, 7, 1, 61), (2, 0, "prims0", 0, 72), (5, 2, "prims1", 0, 50),
    (2, 0, "sierpinski6", 0, 90), (3, 2, "sierpinski4", 0, 64)])
def test_long_ray_pass_matches_twin(gh, budget, lanes, scene, n_prim, n):
    # a small step budget hands nearly every ray to the window pass, which
    # must continue it bit for bit, for every lanes-per-cell split (8 to 64
    # cells per window) and with records in registers or read from LDS (a
    # type group larger than the split)
    native, P = gh
    recs = _named_scene(scene) if isinstance(scene, str) else W.csg_scene(scene, n_prim)
    g = W.grid(n)
    native.gh_set_tuning(hop_lanes_per_ray=lanes, hop_step_budget=budget)
    try:
        out = _run(gh, recs, *g)
    finally:
        native.gh_set_tuning(0)
    ref = ohop.gridhop(osdb.SDB.prims(recs), *g, precision="f32")
    _check_against_twin(out, ref, *[float(x) for x in g])


def test_long_ray_pass_counters_full_size(gh):
    # every budget gives the oracle's exact evaluation and candidate counts
    # at N = 512, repeated runs included
    native, P = gh
    n, lo, h = W.grid(512)
    recs = W.csg_scene(0)
    cells, total, _ = ohop.hop(osdb.SDB.prims(recs), n, lo, h, precision="f32")
    b = P.Bound.prims(recs)
    import torch
    try:
        for budget in (0, 1, 8, 32, 100):
            native.gh_set_tuning(hop_step_budget=budget)
            poly = P.Polygonizer(b, n, lo, h, keep_cells=False)
            for _ in range(2):
                poly.enqueue_hop()
                torch.cuda.synchronize()
                c = P.counters_dict(poly.ctr)
                assert c["n_hop_evals"] == total and c["n_cand"] == len(cells), (budget, c)
    finally:
        native.gh_set_tuning(0)


def test_graph_replay_matches_eager(gh):
    # one captured step (hop or enumeration, then marching cubes), replayed
    # several times with eager work and synchronisations in between: every
    # replay gives that step's eager counters, vertices and triangles bit for
    # bit
    import torch
    native, P = gh
    n, lo, h = W.grid(96)
    poly = P.Polygonizer(P.Bound.prims(W.csg_scene(2)), n, lo, h)
    other = P.Polygonizer(P.Bound.prims(W.csg_scene(4)), *W.grid(40))
    for dense in (False, True):
        ref = poly.run(dense=dense)
        c_ref = dict(ref.counters)
        v_ref, t_ref = ref.verts.clone(), ref.tris.clone()
        poly.capture(dense=dense)
        for rep in range(3):
            poly.verts.zero_()
            poly.tris.zero_()
            poly.replay()
            torch.cuda.synchronize()
            c = P.counters_dict(poly.ctr)
            for k in ("n_hop_evals", "n_cand", "n_corner", "n_cells", "n_vert", "n_tri", "flags"):
                assert c[k] == c_ref[k], (dense, rep, k)
            assert torch.equal(poly.verts[:c["n_vert"]], v_ref) and torch.equal(poly.tris[:c["n_tri"]], t_ref)
            other.run()  # eager work between replays


def test_mesh_repeatable_full_size(gh):
    """The step at full size (CSG-12, N = 512: about 1,000 tiles per scan,
    each publishing its total, building its outputs in LDS, then looking
    back) replayed 50 times from its graph, with eager runs of the same
    step in between: every replay gives the first run's counters, vertices,
    triangles, cells and cases bit for bit."""
    import torch
    native, P = gh
    n, lo, h = W.grid(512)
    poly = P.Polygonizer(P.Bound.prims(W.csg_scene(0)), n, lo, h)
    ref = poly.run()
    c_ref = dict(ref.counters)
    keep = {k: getattr(ref, k).clone() for k in ("verts", "vert_edge", "tris", "cells", "cases")}
    poly.capture()
    for rep in range(50):
        poly.replay()
        if rep % 10 == 9:
            poly.run()  # eager work between replays
        torch.cuda.synchronize()
        c = P.counters_dict(poly.ctr)
        for k in ("n_hop_evals", "n_cand", "n_corner", "n_cells", "n_vert", "n_tri", "flags"):
            assert c[k] == c_ref[k], (rep, k)
        assert torch.equal(poly.verts[:c["n_vert"]], keep["verts"]), rep
        assert torch.equal(poly.vert_edge[:c["n_vert"]], keep["vert_edge"]), rep
        assert torch.equal(poly.tris[:c["n_tri"]], keep["tris"]), rep
        assert torch.equal(poly.cells[:c["n_cells"]], keep["cells"]), rep
        assert torch.equal(poly.cases[:c["n_cells"]], keep["cases"]), rep


def test_csg_n1024_candidates_and_counts(gh):
    # twice the headline size: the candidate cells and every counter of the
    # hop equal the twin's, and the mesh is closed and oriented
    n, lo, h = W.grid(1024)
    recs = W.csg_scene(0)
    out = _run(gh, recs, n, lo, h)
    cells, total, _ = ohop.hop(osdb.SDB.prims(recs), n, lo, h, precision="f32")
    print(f"N=1024 csg0: evals={total} cand={len(cells)} tris={len(out['tris'])}", flush=True)
    assert out["ctr"]["n_hop_evals"] == total and out["ctr"]["n_cand"] == len(cells)
    np.testing.assert_array_equal(out["cand"], cells)
    assert out["ctr"]["n_corner"] == len(ohop.corner_points(n, cells))
    T = np.searchsorted(out["edge"], out["tri_e"])
    assert _closed_oriented(T)


def test_marching_cubes_repeat_after_one_hop(gh):
    """gh_mc keeps its scans clean for the next pass (no clearing launch):
    marching cubes run three times after one hop, the middle time with too
    small a vertex capacity, reproduce the first run exactly, and the
    overflowing run reports the required size."""
    import torch
    native, P = gh
    n, lo, h = W.grid(96)
    poly = P.Polygonizer(P.Bound.prims(W.csg_scene(1)), n, lo, h)
    ref = poly.run()
    keep = {k: getattr(ref, k).clone() for k in ("verts", "vert_edge", "vert_t", "tris", "cells", "cases")}
    c0 = dict(ref.counters)
    for rep in range(3):
        for k in keep:
            getattr(poly, k).fill_(-3 if getattr(poly, k).dtype != torch.float32 else float("nan"))
        small = rep == 1
        st = native.gh_mc(poly.bound.desc, poly.grid, poly.ws, poly.corner_cap, poly.verts, poly.vert_edge,
                          poly.vert_t, 10 if small else poly.vert_cap, poly.tris, poly.tri_cap, poly.cells,
                          poly.cases, poly.cell_cap, poly.ctr)
        native.check(st, "gh_mc")
        torch.cuda.synchronize()
        c = P.counters_dict(poly.ctr)
        print(f"pass {rep}: {c}", flush=True)
        assert c["n_vert"] == c0["n_vert"] and c["n_corner"] == c0["n_corner"]
        if small:
            assert c["flags"] & native.GH_FLAG_CAPACITY
            continue
        assert c == c0
        m = poly.result(c)
        for k, v in keep.items():
            assert torch.equal(getattr(m, k), v), (rep, k)
