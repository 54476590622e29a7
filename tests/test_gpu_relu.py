"""The paper's network shape on the GPU (Section 5.2: eight ReLU layers of
width 64 on the raw coordinates; random weights under the sphere prior and
calibration of the other neural workloads), through the C ABI, against the
FP64 oracle: FP32 values, the bf16 certification taking exactly the FP32
schedule and signs, and meshes against the oracle's."""
import numpy as np
import parity_util as U
import pytest

import workloads as W
from oracle import hop as ohop
from oracle import mesh as omesh
from oracle import sdb as osdb

from test_gpu_mlp import _closed_oriented, _points, _run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05778_amd import native, polygonize
    return native, polygonize


@pytest.fixture(scope="module")
def net():
    return W.paper_net_scene()


def test_fp32_and_bf16_values(gh, net):
    import torch
    native, P = gh
    pts = _points()
    ref = osdb.neural_f64(net, pts.astype(np.float64))
    errs = {}
    for prec in ("fp32", "bf16", "bf16x3"):
        # point values take no decision, so the margin is not used here
        f = P.Bound.mlp(net, prec, margin=None if prec == "fp32" else 1.0).eval(
            torch.from_numpy(pts).cuda()).cpu().numpy().astype(np.float64)
        errs[prec] = np.abs(f - ref).max()
    print("max |f - f64|: " + ", ".join(f"{k} {v:.3e}" for k, v in errs.items()), flush=True)
    assert errs["fp32"] < 2e-5 and errs["bf16x3"] < 1e-4 and errs["bf16"] < 2e-2


@pytest.mark.parametrize("prec,n", [("bf16", 64), ("bf16x3", 77), ("bf16x3", 128)])
def test_bf16_takes_the_fp32_schedule_and_signs(gh, net, prec, n):
    native, P = gh
    margin = P.bf16_margin(net, W.probe_points(seed=3, n=65536), prec)
    g = W.grid(n)
    a = _run(gh, P.Bound.mlp(net, "fp32"), *g)
    b = _run(gh, P.Bound.mlp(net, prec, margin=margin), *g)
    print(f"{prec} n {n}: margin {margin:.2e}, evals {b['ctr']['n_hop_evals']}, re-evaluated {b['ctr']['n_reeval']}",
          flush=True)
    np.testing.assert_array_equal(a["cand"], b["cand"])
    assert a["ctr"]["n_hop_evals"] == b["ctr"]["n_hop_evals"]
    for key in ("cells", "cases", "edge", "tri_e"):
        np.testing.assert_array_equal(a[key], b[key])


@pytest.mark.parametrize("n", [64, 128, 256])
def test_shrunk_bf16_hop_gives_the_fp32_mesh(gh, net, n):
    # plain bf16 with steps of floor(max(|f| - eps, 0)/h) and two-step corner
    # certification: the FP32 path's sign-change cells are all candidates,
    # and cells, cases, edges and triangles are the FP32 path's
    native, P = gh
    probe = W.probe_points(seed=3, n=65536)
    eps, eps3 = P.bf16_margin(net, probe, "bf16"), P.bf16_margin(net, probe, "bf16x3")
    g = W.grid(n)
    a = _run(gh, P.Bound.mlp(net, "fp32"), *g)
    b = _run(gh, P.Bound.mlp(net, "bf16", margin=eps, hop="shrink", margin3=eps3), *g)
    print(f"n {n}: eps {eps:.2e}, hop evals fp32 {a['ctr']['n_hop_evals']} shrink {b['ctr']['n_hop_evals']}, "
          f"candidates {a['ctr']['n_cand']} / {b['ctr']['n_cand']}", flush=True)
    assert b["ctr"]["flags"] == 0
    assert np.all(np.isin(a["cells"], b["cand"]))
    for key in ("cells", "cases", "edge", "tri_e"):
        np.testing.assert_array_equal(a[key], b[key])


@pytest.mark.parametrize("n", [64, 128])
def test_fp32_mesh_matches_fp64_oracle(gh, net, n):
    """The FP32 cells equal the FP64 oracle's once cells with a corner closer
    to zero than four times the measured FP32 error (at least
    max(1e-6 h, 2^-20)) are set aside on both sides."""
    native, P = gh
    _, lo, h = W.grid(n)
    out = _run(gh, P.Bound.mlp(net, "fp32"), n, lo, h)
    ref = ohop.gridhop(osdb.SDB.neural(net), n, lo, h)
    thr = U.fp32_threshold(P, net, n, lo, h, np.union1d(out["cells"], ref.mesh.cells))
    aside = U.assert_cells_match_excluding_near_zero(out["cells"], out["cases"], ref.mesh.cells, ref.mesh.cases,
                                                     lambda X: osdb.neural_f64(net, X), n, lo, h, thr,
                                                     f"relu N={n}")
    assert aside <= 0.01 * len(ref.mesh.cells)
    assert abs(out["ctr"]["n_hop_evals"] - ref.hop_evals) <= 1e-3 * ref.hop_evals


def test_bf16x3_mesh_within_half_cell_of_fp64(gh, net):
    native, P = gh
    n, lo, h = W.grid(64)
    margin = P.bf16_margin(net, W.probe_points(seed=3, n=65536), "bf16x3")
    out = _run(gh, P.Bound.mlp(net, "bf16x3", margin=margin), n, lo, h)
    ref = ohop.gridhop(osdb.SDB.neural(net), n, lo, h).mesh
    T = np.searchsorted(out["edge"], out["tri_e"])
    hd = omesh.hausdorff(out["verts"], T, ref.positions(), ref.tri_vertex_index())
    print(f"Hausdorff {hd:.3e} = {hd / float(h):.4f} h", flush=True)
    assert hd <= 0.5 * float(h)
    assert _closed_oriented(T)


def test_adjoint_refuses_relu(gh, net):
    import torch
    native, P = gh
    from paper_2111_05778_amd.autograd import GridHopMesh, flatten
    n, lo, h = W.grid(16)
    theta = torch.tensor(flatten(net), device="cuda", requires_grad=True)
    with pytest.raises(native.GhError) as e:
        V = GridHopMesh.apply(theta, net, n, float(lo), float(h), "fp32", 0.0)
        V.sum().backward()
    assert e.value.status == native.GH_EUNSUPPORTED
