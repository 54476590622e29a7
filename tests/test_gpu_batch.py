"""Batched polygonization (gh_batch_*) through the C ABI.

A batch runs the hop of every shape in one persistent launch over work items
ordered by estimated cost, then marching cubes per shape.  Only the
scheduling differs from a single-shape run, so per shape every output must
equal the single-shape run bit for bit: all counters, cell ids and case
bytes, welded vertex edge ids, edge parameters t, positions and triangles.
Analytic shapes are also compared with the oracle's float32 twin (same
bar as the single-shape parity tests).  A captured hipGraph is replayed
several times with eager work and synchronisations between the replays, and
every replay is checked against the eager result.
"""
import numpy as np
import parity_util as U
import pytest

import workloads as W
from oracle import hop as ohop
from oracle import mesh as omesh
from oracle import sdb as osdb

pytestmark = pytest.mark.gpu

KEYS = ("verts", "vert_edge", "vert_t", "tris", "cells", "cases")
COUNTERS = ("n_hop_evals", "n_cand", "n_corner", "n_cells", "n_vert", "n_tri", "n_reeval", "flags")


@pytest.fixture(scope="module")
def gh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05778_amd import native, polygonize
    return torch, native, polygonize


def _bound(P, sc, precision, margin_cache):
    if sc["kind"] == "csg":
        return P.Bound.prims(W.csg_scene(sc["seed"], sc["n_prim"]))
    net = W.neural_scene(sc["seed"], sc["width"])
    margin = None

    def measured(prec, with_offset=False):
        key = (sc["seed"], sc["width"], prec, with_offset)
        if key not in margin_cache:
            margin_cache[key] = P.bf16_margin(net, W.probe_points(seed=3, n=65536), prec, with_offset=with_offset)
        return margin_cache[key]

    if precision == "bf16":  # plain bf16: shrunk hop, offset removed, two-step corner certification
        margin, offset = measured("bf16", True)
        return P.Bound.mlp(net, precision, margin=margin, hop="shrink", margin3=measured("bf16x3"), offset=offset)
    if precision != "fp32":
        margin = measured(precision)
    return P.Bound.mlp(net, precision, margin=margin)


def _snap(mesh):
    out = {k: getattr(mesh, k).clone() for k in KEYS}
    out["ctr"] = {k: mesh.counters[k] for k in COUNTERS}
    return out


def _bits(torch, t):
    return t.contiguous().view(-1).view(torch.uint8)


def _assert_same(torch, a, b, label):
    assert a["ctr"] == b["ctr"], f"{label}: counters {a['ctr']} != {b['ctr']}"
    for k in KEYS:
        assert a[k].shape == b[k].shape, f"{label}: {k} shape"
        # raw bytes, so that -0.0 and NaN patterns count too
        assert torch.equal(_bits(torch, a[k]), _bits(torch, b[k])), f"{label}: {k} differs"


def _singles(P, bounds, grids):
    return [_snap(P.Polygonizer(b, *g).run()) for b, g in zip(bounds, grids)]


def _mixed(P, precision, margins, sizes):
    scenes = W.batch_scenes()[:len(sizes)]
    bounds = [_bound(P, sc, precision, margins) for sc in scenes]
    grids = [W.grid(n) for n in sizes]
    return scenes, bounds, grids


# ragged sizes: none of them a multiple of the 8 x 8 hop tile except 64
SIZES = [37, 50, 61, 64, 75, 83, 29, 96]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16"])
def test_mixed_batch_equals_single_runs(gh, precision):
    torch, N, P = gh
    margins = {}
    scenes, bounds, grids = _mixed(P, precision, margins, SIZES)
    single = _singles(P, bounds, grids)
    batch = P.BatchPolygonizer([(b, *g) for b, g in zip(bounds, grids)])
    res = batch.run()
    print(f"{precision}: {len(scenes)} shapes, {batch.item_count()} work items", flush=True)
    for s, (sc, r, ref) in enumerate(zip(scenes, res, single)):
        _assert_same(torch, _snap(r), ref, f"shape {s} {sc['kind']} n={grids[s][0]}")


def test_lean_batch_equals_full_layout(gh):
    # plain bf16 network items on the lean layout (two blocks per CU) and on
    # the full one, read when the batch is created: every output the same
    torch, N, P = gh
    margins = {}
    scenes, bounds, grids = _mixed(P, "bf16", margins, SIZES)
    old = N.gh_get_tuning()
    res = {}
    try:
        for lean in (1, 2):
            N.gh_set_tuning(**{**old, "mlp_lean": lean})
            batch = P.BatchPolygonizer([(b, *g) for b, g in zip(bounds, grids)])
            res[lean] = [_snap(r) for r in batch.run()]
    finally:
        N.gh_set_tuning(**old)
    for s, (a, b) in enumerate(zip(res[1], res[2])):
        _assert_same(torch, a, b, f"shape {s} {scenes[s]['kind']} n={grids[s][0]}")


def test_analytic_batch_matches_twin(gh):
    torch, N, P = gh
    scenes = [sc for sc in W.batch_scenes() if sc["kind"] == "csg"][:6]
    sizes = [41, 64, 23, 90, 57, 70]
    recs = [W.csg_scene(sc["seed"], sc["n_prim"]) for sc in scenes]
    grids = [W.grid(n) for n in sizes]
    batch = P.BatchPolygonizer([(P.Bound.prims(r), *g) for r, g in zip(recs, grids)])
    _check_batch_twin(recs, grids, batch.run())


def test_batch_of_other_families_matches_twin(gh):
    # the paper's seven primitives, the genus-2 surface, Sierpinski
    # tetrahedra and a union of CSG-12 with one, in one launch
    torch, N, P = gh
    recs = [W.primitives_scene(0), W.genus2_scene(), W.sierpinski_scene(4), W.sierpinski_scene(7),
            np.concatenate([W.csg_scene(0), W.sierpinski_scene(5, scale=2.0, centre=(0.31, -0.27, 0.22))])]
    grids = [W.grid(n) for n in (48, 40, 64, 80, 56)]
    batch = P.BatchPolygonizer([(P.Bound.prims(r), *g) for r, g in zip(recs, grids)])
    _check_batch_twin(recs, grids, batch.run())


def _check_batch_twin(recs, grids, res):
    for r, g, m in zip(recs, grids, res):
        n, lo, h = g
        ref = ohop.gridhop(osdb.SDB.prims(r), n, lo, h, precision="f32")
        c = m.counters
        assert c["flags"] == 0
        assert c["n_hop_evals"] == ref.hop_evals
        assert c["n_cand"] == len(ref.candidates)
        assert c["n_corner"] == ref.corner_evals
        np.testing.assert_array_equal(m.cells.cpu().numpy(), ref.mesh.cells)
        np.testing.assert_array_equal(m.cases.cpu().numpy(), ref.mesh.cases)
        np.testing.assert_array_equal(m.vert_edge.cpu().numpy(), ref.mesh.edge_ids)
        if len(ref.mesh.ts):
            assert np.abs(m.vert_t.cpu().numpy().astype(np.float64) - ref.mesh.ts).max() <= 1e-5


def test_graph_replays_equal_eager(gh):
    torch, N, P = gh
    margins = {}
    scenes, bounds, grids = _mixed(P, "bf16x3", margins, [48, 33, 64, 40, 72, 56])
    batch = P.BatchPolygonizer([(b, *g) for b, g in zip(bounds, grids)])
    eager = [_snap(r) for r in batch.run()]
    batch.capture()
    torch.cuda.synchronize()
    other = P.Polygonizer(bounds[0], *W.grid(24))
    for rep in range(4):
        # clobber the outputs and the counters, then run unrelated eager work
        for p in batch.polys:
            p.verts.fill_(float("nan"))
            p.tris.fill_(-1)
            p.ctr.fill_(-1)
        other.run()
        batch.replay()
        torch.cuda.synchronize()
        for s, (p, ref) in enumerate(zip(batch.polys, eager)):
            _assert_same(torch, _snap(p.result()), ref, f"replay {rep} shape {s}")
        x = torch.randn(1 << 20, device="cuda")
        assert torch.isfinite(x.sum())


def test_full_batch_64_shapes(gh):
    # the batched workload: 64 shapes, N in {64, 128, 256, 512}, half CSG
    # unions of 4..16 primitives, half networks of width 64/128/256 (bf16)
    torch, N, P = gh
    margins = {}
    scenes = W.batch_scenes()
    bounds = [_bound(P, sc, "bf16", margins) for sc in scenes]
    grids = [W.grid(sc["n"]) for sc in scenes]
    batch = P.BatchPolygonizer([(b, *g) for b, g in zip(bounds, grids)], keep_cells=True)
    res = [_snap(r) for r in batch.run()]
    single = _singles(P, bounds, grids)
    for s, (a, b) in enumerate(zip(res, single)):
        _assert_same(torch, a, b, f"shape {s} {scenes[s]['kind']} n={grids[s][0]}")
    tot = sum(a["ctr"]["n_tri"] for a in res)
    print(f"64 shapes, {batch.item_count()} items, {tot} triangles", flush=True)
    # the network shapes of the batch at N = 64 (widths 64, 128, 256) against
    # the FP64 oracle: cells under the exclusion rule, mesh within 0.5 h
    for s in (1, 9, 57):
        sc = scenes[s]
        assert sc["kind"] == "mlp" and sc["n"] == 64
        net = W.neural_scene(sc["seed"], sc["width"])
        n, lo, h = grids[s]
        ref = ohop.gridhop(osdb.SDB.neural(net), n, lo, h).mesh
        m = res[s]
        cells, cases = m["cells"].cpu().numpy(), m["cases"].cpu().numpy()
        f64 = lambda X: osdb.neural_f64(net, X)  # noqa: E731
        # corner signs are certified FP32 signs, so the FP32 error sets the threshold
        thr = U.fp32_threshold(P, net, n, lo, h, np.union1d(cells, ref.cells))
        U.assert_cells_match_excluding_near_zero(cells, cases, ref.cells, ref.cases, f64, n, lo, h, thr,
                                                 f"batch shape {s} width {sc['width']}")
        V = m["verts"].cpu().numpy().astype(np.float64)
        T = m["tris"].cpu().numpy().astype(np.int64)
        hd = omesh.hausdorff(V, T, ref.positions(), ref.tri_vertex_index())
        print(f"batch shape {s}: Hausdorff to FP64 {hd / float(h):.4f} h", flush=True)
        assert hd <= 0.5 * float(h)


def test_batch_rejects_mixed_network_precisions(gh):
    torch, N, P = gh
    scenes = [sc for sc in W.batch_scenes() if sc["kind"] == "mlp"][:2]
    b0 = P.Bound.mlp(W.neural_scene(scenes[0]["seed"], scenes[0]["width"]), "fp32")
    b1 = P.Bound.mlp(W.neural_scene(scenes[1]["seed"], scenes[1]["width"]), "bf16", margin=1e-2)
    with pytest.raises(N.GhError) as e:
        P.BatchPolygonizer([(b0, *W.grid(32)), (b1, *W.grid(32))])
    assert e.value.status == N.GH_EUNSUPPORTED
