"""The launch-shape autotuner on the device: every candidate reproduces the
reference mesh (the shapes change the time only), the winner is cached per
device and workload, and a Polygonizer with tuning="auto" picks it up."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05778_amd import autotune, native, polygonize
    return torch, native, polygonize, autotune


def test_tune_analytic_and_reuse(gh, tmp_path, monkeypatch):
    torch, N, P, A = gh
    path = str(tmp_path / "tune.json")
    monkeypatch.setenv("GH_AUTOTUNE_CACHE", path)
    bound = P.Bound.prims(W.csg_scene(0))
    poly = P.Polygonizer(bound, *W.grid(96))
    ref = poly.run()
    ref_tris = ref.tris.clone()
    best, ms, trials = A.tune(poly, reps=2)
    print("analytic:", best, f"{ms:.3f} ms", [(t, m) for t, m in trials], flush=True)
    assert all(m is not None for _, m in trials)  # no candidate changed the mesh
    assert A.lookup(A.signature(bound.spec, 96)) == best
    auto = P.Polygonizer(bound, *W.grid(96), tuning="auto")
    assert auto.tuning == best
    m = auto.run()
    assert torch.equal(m.tris, ref_tris)
    assert N.gh_get_tuning() == A.full(best)
    N.gh_set_tuning()


@pytest.mark.parametrize("prec,hop", [("bf16x3", "fp32"), ("bf16", "shrink")])
def test_tune_network(gh, tmp_path, prec, hop):
    # every candidate, the ray pool and tail windows included, must reproduce
    # the reference counters and triangles bit for bit
    torch, N, P, A = gh
    net = W.neural_scene(0, 64)
    probe = W.probe_points(seed=3, n=65536)
    margin = P.bf16_margin(net, probe, prec)
    margin3 = P.bf16_margin(net, probe, "bf16x3") if prec == "bf16" else 0.0
    poly = P.Polygonizer(P.Bound.mlp(net, prec, margin=margin, hop=hop, margin3=margin3), *W.grid(48))
    poly.run()
    best, ms, trials = A.tune(poly, reps=1, path=str(tmp_path / "t.json"))
    print("network:", best, [(t, m) for t, m in trials], flush=True)
    assert all(m is not None for _, m in trials)
    N.gh_set_tuning()


def test_tune_batch(gh, tmp_path):
    torch, N, P, A = gh
    scenes = W.batch_scenes()[:4]
    margin = {}
    items = []
    for sc, n in zip(scenes, (40, 56, 33, 64)):
        if sc["kind"] == "csg":
            b = P.Bound.prims(W.csg_scene(sc["seed"], sc["n_prim"]))
        else:
            net = W.neural_scene(sc["seed"], sc["width"])
            b = P.Bound.mlp(net, "bf16x3", margin=P.bf16_margin(net, W.probe_points(seed=3, n=65536), "bf16x3"))
        items.append((b, n))

    def make():
        return P.BatchPolygonizer([(b, *W.grid(n)) for b, n in items])

    best, ms, trials = A.tune_batch(make, items, reps=1, space={"batch_rays_per_item": [256, 1024, 4096]},
                                    path=str(tmp_path / "b.json"))
    print("batch:", best, [(t, m) for t, m in trials], flush=True)
    assert all(m is not None for _, m in trials)
    assert A.load_cache(str(tmp_path / "b.json"))
    N.gh_set_tuning()
