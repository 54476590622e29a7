"""GPU parity of the neural bound (eq. nnsdb with the sphere prior) against
the FP64 oracle, through the C ABI.

* FP32 evaluator (MFMA f32): values within 2e-5 of FP64; the FP32 mesh has
  the oracle's sign-change cells once cells with a corner closer to zero
  than four times the measured FP32 error are set aside (count reported).
* bf16 evaluators (MFMA bf16, FP32 accumulation; plain and hi/lo split):
  with the measured margin eps the hop takes exactly the FP32 schedule and
  every corner sign is the FP32 sign (ambiguous values are re-evaluated in
  FP32), so cells, cases and triangles equal the FP32 path's; the vertices
  differ only through t.
* bf16 meshes within 0.5 h (Hausdorff) of the FP64 oracle's mesh.
* Full size (N = 256 and 512, width 256), on a band of ray-column rows
  through the middle of the shape that the FP64 oracle computes: the FP32
  cells equal the oracle's under the exclusion rule, and the bf16 and bf16x3
  meshes lie within 0.5 h of the oracle's (Hausdorff).
* Full size N = 512, width 256, split bf16: the FP32 schedule and signs, a
  closed oriented mesh, and every vertex on the FP64 surface to within a
  quarter cell.
"""
import numpy as np
import parity_util as U
import pytest

import workloads as W
from oracle import hop as ohop
from oracle import mc as omc
from oracle import mesh as omesh
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
    r = np.argmin(tri_e, axis=1)
    t = np.take_along_axis(tri_e, (r[:, None] + np.arange(3)) % 3, axis=1)
    return t[np.lexsort((t[:, 2], t[:, 1], t[:, 0]))]


def _run(gh, bound, n, lo, h, dense=False):
    native, P = gh
    poly = P.Polygonizer(bound, n, lo, h)
    m = poly.run(dense=dense)
    out = {"cand": poly.candidates().cpu().numpy(), "ctr": m.counters,
           "verts": m.verts.cpu().numpy().astype(np.float64), "edge": m.vert_edge.cpu().numpy(),
           "tris": m.tris.cpu().numpy().astype(np.int64), "cells": m.cells.cpu().numpy(),
           "cases": m.cases.cpu().numpy()}
    out["tri_e"] = _canon(out["edge"][out["tris"]]) if len(out["tris"]) else np.zeros((0, 3), np.int64)
    return out


def _closed_oriented(tris):
    v = int(tris.max()) + 1
    d = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    key = d[:, 0] * v + d[:, 1]
    return len(np.unique(key)) == len(key) and np.isin(d[:, 1] * v + d[:, 0], key).all()


def _points(n=20000, seed=5):
    return np.random.default_rng(seed).uniform(-1, 1, (n, 3)).astype(np.float32)


@pytest.mark.parametrize("width", [64, 128, 256])
def test_fp32_values_match_fp64(gh, width):
    import torch
    native, P = gh
    net = W.neural_scene(0, width)
    pts = _points()
    f = P.Bound.mlp(net, "fp32").eval(torch.from_numpy(pts).cuda()).cpu().numpy().astype(np.float64)
    ref = osdb.neural_f64(net, pts.astype(np.float64))
    err = np.abs(f - ref).max()
    print(f"width {width}: max |f32 - f64| = {err:.3e}", flush=True)
    assert err < 2e-5


@pytest.mark.parametrize("width", [64, 256])
def test_bf16_values_close_to_fp64(gh, width):
    import torch
    native, P = gh
    net = W.neural_scene(0, width)
    pts = _points()
    ref = osdb.neural_f64(net, pts.astype(np.float64))
    errs = {}
    for prec in ("bf16", "bf16x3"):
        # point values take no decision, so the margin is not used here
        f = P.Bound.mlp(net, prec, margin=1.0).eval(torch.from_numpy(pts).cuda()).cpu().numpy().astype(np.float64)
        errs[prec] = np.abs(f - ref).max()
    m3 = P.bf16_margin(net, W.probe_points(seed=3, n=65536), "bf16x3")
    print(f"width {width}: max |f - f64| bf16 {errs['bf16']:.3e}, bf16x3 {errs['bf16x3']:.3e}; "
          f"bf16x3 margin {m3:.3e}", flush=True)
    assert errs["bf16"] < 2e-2
    # the split keeps the margin far below the 0.134 h guard of the hop rule at N = 512
    assert errs["bf16x3"] < 1e-4 and m3 < 0.05 * 0.134 * (2.0 / 512)


@pytest.mark.parametrize("width,n", [(64, 64), (256, 48), (64, 37)])
def test_fp32_mesh_matches_fp64_oracle(gh, width, n):
    import torch
    native, P = gh
    net = W.neural_scene(0, width)
    g = W.grid(n)
    out = _run(gh, P.Bound.mlp(net, "fp32"), *g)
    ref = ohop.gridhop(osdb.SDB.neural(net), *g)
    # exclusion threshold from the measured FP32 error at the oracle's corners
    pid = ohop.corner_points(n, ref.candidates)
    n1 = n + 1
    a, b, c = pid // (n1 * n1), (pid // n1) % n1, pid % n1
    P64 = np.stack([omc.lattice_coords_f64(n, g[1], g[2], v) for v in (a, b, c)], axis=1)
    f64 = osdb.neural_f64(net, P64)
    f32 = P.Bound.mlp(net, "fp32").eval(torch.from_numpy(P64.astype(np.float32)).cuda()).cpu().numpy()
    thr = max(1e-6 * float(g[2]), 2.0 ** -20, 4 * np.abs(f32 - f64).max())
    near_pid = set(pid[np.abs(f64) < thr].tolist())

    def near(cells):
        out_ = []
        for cell in cells:
            i, j, k = cell // (n * n), (cell // n) % n, cell % n
            ids = [((i + dx) * n1 + (j + dy)) * n1 + (k + dz) for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)]
            out_.append(any(q in near_pid for q in ids))
        return np.array(out_, dtype=bool)

    ga, oa = out["cells"], ref.mesh.cells
    print(f"width {width} n {n}: thr {thr:.2e}, gpu cells {len(ga)}, oracle {len(oa)}, "
          f"excluded {int(near(ga).sum())}/{int(near(oa).sum())}", flush=True)
    np.testing.assert_array_equal(ga[~near(ga)], oa[~near(oa)])
    # evaluation counts agree up to float rounding at floor() boundaries
    assert abs(out["ctr"]["n_hop_evals"] - ref.hop_evals) <= 1e-3 * ref.hop_evals


@pytest.mark.parametrize("prec,width,n", [("bf16", 256, 64), ("bf16", 64, 128), ("bf16x3", 128, 96),
                                          ("bf16x3", 256, 128), ("bf16x3", 64, 77), ("bf16x3", 256, 512)])
def test_bf16_takes_the_fp32_schedule_and_signs(gh, prec, width, n):
    native, P = gh
    net = W.neural_scene(0, width)
    margin = P.bf16_margin(net, W.probe_points(seed=3, n=65536), prec)
    g = W.grid(n)
    a = _run(gh, P.Bound.mlp(net, "fp32"), *g)
    b = _run(gh, P.Bound.mlp(net, prec, margin=margin), *g)
    print(f"{prec} width {width} n {n}: margin {margin:.2e}, evals {b['ctr']['n_hop_evals']}, "
          f"re-evaluated {b['ctr']['n_reeval']}", flush=True)
    np.testing.assert_array_equal(a["cand"], b["cand"])
    assert a["ctr"]["n_hop_evals"] == b["ctr"]["n_hop_evals"]
    for key in ("cells", "cases", "edge", "tri_e"):
        np.testing.assert_array_equal(a[key], b[key])


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
def test_bf16_mesh_within_half_cell_of_fp64(gh, prec):
    native, P = gh
    net = W.neural_scene(0, 256)
    n, lo, h = W.grid(64)
    margin = P.bf16_margin(net, W.probe_points(seed=3, n=65536), prec)
    out = _run(gh, P.Bound.mlp(net, prec, margin=margin), n, lo, h)
    ref = ohop.gridhop(osdb.SDB.neural(net), n, lo, h).mesh
    T = np.searchsorted(out["edge"], out["tri_e"])
    hd = omesh.hausdorff(out["verts"], T, ref.positions(), ref.tri_vertex_index())
    print(f"{prec}: Hausdorff {hd:.3e} = {hd / float(h):.4f} h", flush=True)
    assert hd <= 0.5 * float(h)
    assert _closed_oriented(T)


def test_bf16_dense_equals_hop(gh):
    native, P = gh
    net = W.neural_scene(0, 64)
    g = W.grid(48)
    margin = P.bf16_margin(net, W.probe_points(seed=3, n=65536))
    bnd = P.Bound.mlp(net, "bf16", margin=margin)
    a, b = _run(gh, bnd, *g), _run(gh, bnd, *g, dense=True)
    for key in ("cells", "cases", "edge", "tri_e"):
        np.testing.assert_array_equal(a[key], b[key])
    assert b["ctr"]["n_hop_evals"] == 49 ** 3


def test_full_size_bf16x3_n512(gh):
    native, P = gh
    net = W.neural_scene(0, 256)
    n, lo, h = W.grid(512)
    margin = P.bf16_margin(net, W.probe_points(seed=3, n=65536), "bf16x3")
    out = _run(gh, P.Bound.mlp(net, "bf16x3", margin=margin), n, lo, h)
    c = out["ctr"]
    print(f"N=512 neural bf16x3 margin {margin:.2e}: {c}", flush=True)
    T = np.searchsorted(out["edge"], out["tri_e"])
    assert _closed_oriented(T)
    f = osdb.neural_f64(net, out["verts"])          # every vertex
    print(f"max |f64| at the vertices {np.abs(f).max():.2e} = {np.abs(f).max() / float(h):.4f} h", flush=True)
    assert np.abs(f).max() <= 0.25 * float(h)
    assert c["n_reeval"] < 0.01 * c["n_hop_evals"]


# Rows i of ray columns through the middle of the shape, one sixteenth or one
# thirty-second of the grid: the FP64 oracle's hop on these columns alone
# takes seconds, where the whole grid takes minutes.
BANDS = {256: (120, 136), 512: (248, 264)}
_ORACLE_BANDS = {}


def _oracle_band(net, n):
    if n not in _ORACLE_BANDS:
        _, lo, h = W.grid(n)
        _ORACLE_BANDS[n] = U.oracle_band(osdb.SDB.neural(net), n, lo, h, *BANDS[n]).mesh
    return _ORACLE_BANDS[n]


@pytest.mark.parametrize("n", [256, 512])
def test_full_size_fp32_cells_match_fp64_on_a_band(gh, n):
    native, P = gh
    net = W.neural_scene(0, 256)
    _, lo, h = W.grid(n)
    out = _run(gh, P.Bound.mlp(net, "fp32"), n, lo, h)
    ref = _oracle_band(net, n)
    cells, cases, _, _ = U.gpu_band(out["cells"], out["cases"], out["verts"], out["tris"], n, *BANDS[n])
    thr = U.fp32_threshold(P, net, n, lo, h, np.union1d(cells, ref.cells))
    aside = U.assert_cells_match_excluding_near_zero(cells, cases, ref.cells, ref.cases,
                                                     lambda X: osdb.neural_f64(net, X), n, lo, h, thr,
                                                     f"N={n} band rows {BANDS[n]}")
    assert aside <= 0.01 * len(ref.cells)


@pytest.mark.parametrize("prec,n", [("bf16x3", 256), ("bf16", 256), ("bf16x3", 512), ("bf16", 512)])
def test_full_size_bf16_mesh_within_half_cell_on_a_band(gh, prec, n):
    native, P = gh
    net = W.neural_scene(0, 256)
    _, lo, h = W.grid(n)
    margin = P.bf16_margin(net, W.probe_points(seed=3, n=65536), prec)
    out = _run(gh, P.Bound.mlp(net, prec, margin=margin), n, lo, h)
    ref = _oracle_band(net, n)
    _, _, V, T = U.gpu_band(out["cells"], out["cases"], out["verts"], out["tris"], n, *BANDS[n])
    hd = omesh.hausdorff(V, T, ref.positions(), ref.tri_vertex_index())
    print(f"{prec} N={n} band {BANDS[n]}: {len(T)} triangles, Hausdorff {hd:.3e} = {hd / float(h):.4f} h",
          flush=True)
    assert len(T) > 0 and hd <= 0.5 * float(h)


@pytest.mark.parametrize("prec,width", [("bf16", 64), ("bf16", 256), ("bf16x3", 128), ("bf16x3", 256)])
def test_value_does_not_depend_on_tile_fill(gh, prec, width):
    # tiles with few rows spread their layers over more waves; the value of a
    # point must be the same bits whatever else shares its tile
    import torch
    native, P = gh
    net = W.neural_scene(0, width)
    b = P.Bound.mlp(net, prec, margin=1e-3)
    pts = torch.tensor(W.probe_points(seed=11, n=300).astype(np.float32), device="cuda")
    full = b.eval(pts).cpu().numpy()
    for n in (1, 5, 31, 32, 33, 64, 65, 100, 127, 128, 129):
        part = b.eval(pts[:n].contiguous()).cpu().numpy()
        np.testing.assert_array_equal(part.view(np.uint32), full[:n].view(np.uint32), err_msg=f"n={n}")


@pytest.mark.parametrize("prec,width,n", [("bf16", 64, 77), ("bf16", 128, 100), ("bf16", 256, 128),
                                          ("bf16", 256, 512), ("bf16x3", 256, 512)])
def test_shrunk_bf16_hop_gives_the_fp32_mesh(gh, prec, width, n):
    """The bf16 hop without FP32 re-evaluation (steps of
    floor(max(|f| - eps, 0)/h)): every sign-change cell of the FP32 path is a
    candidate, and since corner signs stay certified the cells, cases, edges
    and triangles are the FP32 path's; only the counts differ."""
    native, P = gh
    net = W.neural_scene(0, width)
    margin = P.bf16_margin(net, W.probe_points(seed=3, n=65536), prec)
    g = W.grid(n)
    a = _run(gh, P.Bound.mlp(net, "fp32"), *g)
    b = _run(gh, P.Bound.mlp(net, prec, margin=margin, hop="shrink"), *g)
    ca, cb = a["ctr"], b["ctr"]
    print(f"{prec} w{width} N={n} margin {margin:.2e} = {margin / float(g[2]):.3f} h: hop evals fp32 "
          f"{ca['n_hop_evals']} shrink {cb['n_hop_evals']}, candidates {ca['n_cand']} / {cb['n_cand']}, "
          f"re-evaluated {cb['n_reeval']}", flush=True)
    assert cb["flags"] == 0
    assert np.all(np.isin(a["cells"], b["cand"]))
    for key in ("cells", "cases", "edge", "tri_e"):
        np.testing.assert_array_equal(a[key], b[key])
    assert cb["n_hop_evals"] >= 0.9 * ca["n_hop_evals"]


@pytest.mark.parametrize("width,n", [(64, 77), (128, 100), (256, 128), (256, 512), ("paper", 77)])
def test_lean_layout_changes_nothing(gh, width, n):
    # the shrunk plain bf16 hop and the corner values on the lean layout (two
    # blocks per CU, at width 256 every tile split over two waves per group,
    # corner signs certified in a pass of their own) and on the full layout:
    # the same counters, candidates, vertices and triangles
    # ("paper": the 8 x 64 ReLU network, whose width-64 kernels keep the
    # weights resident and apply max(z, 0) alone)
    native, P = gh
    net = W.paper_net_scene() if width == "paper" else W.neural_scene(0, width)
    probe = W.probe_points(seed=3, n=65536)
    b = P.Bound.mlp(net, "bf16", margin=P.bf16_margin(net, probe, "bf16"), hop="shrink",
                    margin3=P.bf16_margin(net, probe, "bf16x3"))
    g = W.grid(n)
    old = native.gh_get_tuning()
    try:
        native.gh_set_tuning(**{**old, "mlp_lean": 1})
        lean = _run(gh, b, *g)
        native.gh_set_tuning(**{**old, "mlp_lean": 2})
        full = _run(gh, b, *g)
    finally:
        native.gh_set_tuning(**old)
    assert lean["ctr"] == full["ctr"] and lean["ctr"]["flags"] == 0
    for key in ("cand", "cells", "cases", "edge", "tris"):
        np.testing.assert_array_equal(lean[key], full[key])
    np.testing.assert_array_equal(lean["verts"].view(np.uint64), full["verts"].view(np.uint64))


@pytest.mark.parametrize("width,n", [(64, 77), (256, 128), (256, 512)])
def test_offset_removed_from_bf16_values(gh, width, n):
    """Plain bf16 with the measured offset of its error removed: the margin of
    the offset values is at most the plain one, |f_bf16 - offset - f_fp32|
    stays within it on other points, and the shrunk hop with two-step
    signs still gives the FP32 path's cells, cases, edges and triangles."""
    import torch
    native, P = gh
    net = W.neural_scene(0, width)
    probe = W.probe_points(seed=3, n=65536)
    eps_plain = P.bf16_margin(net, probe, "bf16")
    eps, off = P.bf16_margin(net, probe, "bf16", with_offset=True)
    eps3 = P.bf16_margin(net, probe, "bf16x3")
    print(f"w{width}: margin {eps_plain:.3e} plain, {eps:.3e} after the offset {off:.3e}", flush=True)
    assert 0 < eps <= eps_plain
    b = P.Bound.mlp(net, "bf16", margin=eps, hop="shrink", margin3=eps3, offset=off)
    pts = torch.tensor(_points(20000, seed=8), device="cuda")
    f32 = P.Bound.mlp(net, "fp32").eval(pts).cpu().numpy().astype(np.float64)
    fb = b.eval(pts).cpu().numpy().astype(np.float64)
    assert np.abs(fb - f32).max() <= eps
    g = W.grid(n)
    a = _run(gh, P.Bound.mlp(net, "fp32"), *g)
    c = _run(gh, b, *g)
    assert c["ctr"]["flags"] == 0 and np.all(np.isin(a["cells"], c["cand"]))
    for key in ("cells", "cases", "edge", "tri_e"):
        np.testing.assert_array_equal(a[key], c[key])


@pytest.mark.parametrize("n", [128, 512])
def test_two_step_corner_certification(gh, n):
    """Plain bf16 with the split form's margin eps3: corner values within eps
    of zero are certified by a split-bf16 value first and go to FP32 only
    within eps3 of zero.  The cells, cases, edges and triangles stay the FP32
    path's, the mesh stays within 0.5 h of it (surface Hausdorff on the band
    of rows through the shape), and far fewer values need FP32."""
    import torch
    native, P = gh
    net = W.neural_scene(0, 256)
    probe = W.probe_points(seed=3, n=65536)
    eps, eps3 = P.bf16_margin(net, probe, "bf16"), P.bf16_margin(net, probe, "bf16x3")
    g = W.grid(n)
    a = _run(gh, P.Bound.mlp(net, "fp32"), *g)
    one = _run(gh, P.Bound.mlp(net, "bf16", margin=eps, hop="shrink"), *g)
    two = _run(gh, P.Bound.mlp(net, "bf16", margin=eps, hop="shrink", margin3=eps3), *g)
    print(f"N={n}: eps {eps:.2e} eps3 {eps3:.2e}; FP32 re-evaluations one step {one['ctr']['n_reeval']}, "
          f"two steps {two['ctr']['n_reeval']}", flush=True)
    for key in ("cells", "cases", "edge", "tri_e"):
        np.testing.assert_array_equal(a[key], two[key])
    i0, i1 = n // 2 - 8, n // 2 + 8
    _, _, VA, TA = U.gpu_band(a["cells"], a["cases"], a["verts"], a["tris"], n, i0, i1)
    _, _, VB, TB = U.gpu_band(two["cells"], two["cases"], two["verts"], two["tris"], n, i0, i1)
    hd = omesh.hausdorff(VB, TB, VA, TA)
    print(f"N={n}: Hausdorff to the FP32 mesh on rows {i0}..{i1}: {hd / float(g[2]):.4f} h", flush=True)
    assert hd <= 0.5 * float(g[2])
    assert two["ctr"]["n_reeval"] < 0.1 * one["ctr"]["n_reeval"]
    assert two["ctr"]["n_hop_evals"] == one["ctr"]["n_hop_evals"]
