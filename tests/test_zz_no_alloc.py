"""gh_polygonize_noalloc (gh_hop + gh_mc on the library's fixed workspace,
no allocation) against gh_hop + gh_mc on a caller workspace, through the C
ABI: the same counters and bit-identical outputs on two calls in a row, the
second on a smaller grid, for an analytic bound and network bounds (FP32,
and plain bf16 on the lean kernels)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05778_amd import native, polygonize
    return torch, native, polygonize


def _host(m, ctr):
    nv, nt, nc = ctr["n_vert"], ctr["n_tri"], ctr["n_cells"]
    return {"verts": m["verts"][:nv].cpu().numpy(), "edge": m["edge"][:nv].cpu().numpy(),
            "t": m["t"][:nv].cpu().numpy(), "tris": m["tris"][:nt].cpu().numpy(),
            "cells": m["cells"][:nc].cpu().numpy(), "cases": m["cases"][:nc].cpu().numpy()}


def _reference(gh, bound, n, lo, h):
    torch, N, P = gh
    poly = P.Polygonizer(bound, n, lo, h)
    m = poly.run()
    c = dict(m.counters)
    out = _host({"verts": m.verts, "edge": m.vert_edge, "t": m.vert_t, "tris": m.tris, "cells": m.cells,
                 "cases": m.cases}, c)
    return poly, c, out


def _noalloc(gh, bound, n, lo, h, corner_cap, vert_cap, tri_cap, cell_cap):
    torch, N, P = gh
    dev = "cuda"
    # outputs filled with garbage: every value compared must be written by the call
    bufs = {"verts": torch.full((vert_cap, 3), -7.0, dtype=torch.float32, device=dev),
            "edge": torch.full((vert_cap,), -7, dtype=torch.int64, device=dev),
            "t": torch.full((vert_cap,), -7.0, dtype=torch.float32, device=dev),
            "tris": torch.full((tri_cap, 3), -7, dtype=torch.int32, device=dev),
            "cells": torch.full((cell_cap,), -7, dtype=torch.int64, device=dev),
            "cases": torch.full((cell_cap,), 77, dtype=torch.uint8, device=dev)}
    ctr = torch.full((8,), -1, dtype=torch.int64, device=dev)
    grid = N.make_grid(n, lo, h)
    N.check(N.gh_polygonize_noalloc(bound.desc, grid, corner_cap, bufs["verts"], bufs["edge"], bufs["t"], vert_cap,
                                    bufs["tris"], tri_cap, bufs["cells"], bufs["cases"], cell_cap, ctr),
            "gh_polygonize_noalloc")
    torch.cuda.synchronize()
    c = P.counters_dict(ctr)
    return c, _host(bufs, c)


def _same(c_ref, ref, c, got, label):
    print(f"{label}: {c}", flush=True)
    assert c == c_ref, (label, c, c_ref)
    assert c["flags"] == 0
    for k in ref:
        np.testing.assert_array_equal(got[k], ref[k], err_msg=f"{label}: {k}")


def test_noalloc_equals_hop_and_mc_twice(gh):
    torch, N, P = gh
    cases = [("csg12 n=128", W.csg_scene(0), 128, True), ("sphere n=48", W.sphere_scene(), 48, False)]
    for label, recs, n, explicit_cap in cases:   # the second call is smaller and uses the automatic capacity
        _, lo, h = W.grid(n)
        bound = P.Bound.prims(recs)
        poly, c_ref, ref = _reference(gh, bound, n, lo, h)
        cap = poly.corner_cap if explicit_cap else 0
        c, got = _noalloc(gh, bound, n, lo, h, cap, poly.vert_cap, poly.tri_cap, poly.cell_cap)
        _same(c_ref, ref, c, got, label)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_network_twice(gh, prec):
    # plain bf16 takes the shrunk hop and the lean kernels, with two-step
    # certified corner signs
    torch, N, P = gh
    width = 64 if prec == "fp32" else 256
    net = W.neural_scene(0, width)
    if prec == "fp32":
        bound = P.Bound.mlp(net, "fp32")
    else:
        probe = W.probe_points(seed=3, n=65536)
        bound = P.Bound.mlp(net, "bf16", margin=P.bf16_margin(net, probe, "bf16"), hop="shrink",
                            margin3=P.bf16_margin(net, probe, "bf16x3"))
    for n in (40, 24):
        _, lo, h = W.grid(n)
        poly, c_ref, ref = _reference(gh, bound, n, lo, h)
        c, got = _noalloc(gh, bound, n, lo, h, 0, poly.vert_cap, poly.tri_cap, poly.cell_cap)
        _same(c_ref, ref, c, got, f"network {prec} w{width} n={n}")


def test_noalloc_refuses_a_grid_beyond_the_fixed_workspace(gh):
    torch, N, P = gh
    bound = P.Bound.prims(W.sphere_scene())
    ctr = torch.full((8,), -1, dtype=torch.int64, device="cuda")
    for n, cap in ((1024, 0), (512, 10_000_000)):
        _, lo, h = W.grid(n)
        st = N.gh_polygonize_noalloc(bound.desc, N.make_grid(n, lo, h), cap, None, None, None, 0, None, 0, None,
                                     None, 0, ctr)
        assert st == N.GH_ECAPACITY, st
        assert b"fixed workspace" in N.lib.gh_last_error()
    torch.cuda.synchronize()
    assert (ctr.cpu() == -1).all()      # nothing was enqueued
