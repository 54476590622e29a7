"""Host-side parts of the launch-shape autotuner and of gh_set_tuning (no GPU)."""
import ctypes

import numpy as np
import pytest

import workloads as W
from paper_2111_05778_amd import autotune as A
from paper_2111_05778_amd import native as N


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "cache.json")
    assert A.load_cache(path) == {}
    A.save_cache({"dev": {"k": {"hop_lanes_per_ray": 2}}}, path)
    assert A.load_cache(path) == {"dev": {"k": {"hop_lanes_per_ray": 2}}}
    (tmp_path / "bad.json").write_text("{not json")
    assert A.load_cache(str(tmp_path / "bad.json")) == {}


def test_full_resolves_zero_and_missing_to_defaults():
    t = A.full({"hop_lanes_per_ray": 0, "scan_blocks_per_cu": 8, "unknown": 3})
    assert t == dict(A.DEFAULTS, scan_blocks_per_cu=8)
    assert A.full({"hop_lanes_per_ray": 3})["hop_lanes_per_ray"] == 3


def test_coordinate_descent_finds_the_minimum_and_skips_wrong_results():
    cost = {("hop_lanes_per_ray", 1): -1.0, ("hop_lanes_per_ray", 2): -3.0, ("hop_lanes_per_ray", 8): -5.0,
            ("scan_blocks_per_cu", 2): -1.0, ("scan_blocks_per_cu", 8): 2.0}

    def measure(t):
        ms = 10.0 + sum(v for (k, x), v in cost.items() if t[k] == x)
        ok = t["hop_lanes_per_ray"] != 8  # a candidate that changes the result is discarded
        return ms, ok

    space = {"hop_lanes_per_ray": [1, 2, 4, 8], "scan_blocks_per_cu": [1, 2, 4, 8]}
    best, ms, trials = A.coordinate_descent(space, measure)
    assert best["hop_lanes_per_ray"] == 2 and best["scan_blocks_per_cu"] == 2
    assert ms == pytest.approx(6.0)
    assert any(t["hop_lanes_per_ray"] == 8 and m is None for t, m in trials)


def test_coordinate_descent_refuses_a_wrong_start():
    with pytest.raises(RuntimeError):
        A.coordinate_descent({"mlp_split": [1, 2]}, lambda t: (1.0, False))


def test_signature_depends_on_shape_not_values():
    def spec_of(recs):
        rec = np.ascontiguousarray(np.asarray(recs, dtype=np.float32).reshape(-1, N.GH_PRIM_FLOATS))
        sp = N.gh_sdb_spec()
        sp.kind = N.GH_SDB_PRIMS
        sp.n_prim = rec.shape[0]
        sp.prims_h = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        return sp, rec

    a, ka = spec_of(W.csg_scene(0, 12))
    b, kb = spec_of(W.csg_scene(1, 12))
    c, kc = spec_of(W.csg_scene(0, 8))
    assert A.signature(a, 256) == A.signature(b, 256) == "prims:3-3-3-3-0-0-0-0-0-0-0:n256"
    assert A.signature(a, 256) != A.signature(c, 256) and A.signature(a, 256) != A.signature(a, 512)


def _spec_of(recs):
    rec = np.ascontiguousarray(np.asarray(recs, dtype=np.float32).reshape(-1, N.GH_PRIM_FLOATS))
    sp = N.gh_sdb_spec()
    sp.kind = N.GH_SDB_PRIMS
    sp.n_prim = rec.shape[0]
    sp.prims_h = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    return sp, rec


def test_signature_counts_every_record_type():
    """One record of each of the library's types, as in the seven-primitive,
    genus-2 and fractal scenes; an unknown type is refused."""
    recs = np.zeros((N.GH_PRIM_TYPES, N.GH_PRIM_FLOATS), np.float32)
    recs[:, 0] = np.arange(N.GH_PRIM_TYPES)
    sp, keep = _spec_of(recs)
    assert A.signature(sp, 64) == "prims:" + "-".join(["1"] * N.GH_PRIM_TYPES) + ":n64"
    for scene in (W.primitives_scene(0), W.genus2_scene(), W.sierpinski_scene(4)):
        sp, keep = _spec_of(scene)
        assert A.signature(sp, 128).startswith("prims:")
    recs[3, 0] = N.GH_PRIM_TYPES
    sp, keep = _spec_of(recs)
    with pytest.raises(ValueError):
        A.signature(sp, 64)


def test_set_tuning_validates_and_round_trips():
    old = N.gh_get_tuning()
    try:
        N.gh_set_tuning(hop_lanes_per_ray=2, scan_blocks_per_cu=8, batch_rays_per_item=1024, mlp_split=1,
                        mc_items_per_thread=2, hop_step_budget=48, mlp_pool_tiles=1, mlp_spec_rows=8,
                        mlp_lean=2)
        assert N.gh_get_tuning() == {"hop_lanes_per_ray": 2, "scan_blocks_per_cu": 8,
                                     "batch_rays_per_item": 1024, "mlp_split": 1, "mc_items_per_thread": 2,
                                     "hop_step_budget": 48, "mlp_pool_tiles": 1, "mlp_spec_rows": 8,
                                     "mlp_lean": 2}
        for bad in ({"hop_lanes_per_ray": 5}, {"scan_blocks_per_cu": 16}, {"batch_rays_per_item": 1000},
                    {"batch_rays_per_item": 128}, {"mlp_split": 4}, {"mlp_split": -1},
                    {"mc_items_per_thread": 3}, {"hop_step_budget": -1}, {"hop_step_budget": 4097},
                    {"mlp_pool_tiles": 3}, {"mlp_spec_rows": 4}, {"mlp_spec_rows": 64},
                    {"mlp_lean": 3}, {"mlp_lean": -1}):
            with pytest.raises(N.GhError):
                N.gh_set_tuning(**bad)
        t = N.gh_tuning()
        t.reserved = 1
        assert N.lib.gh_set_tuning(ctypes.byref(t)) == N.GH_EINVAL
    finally:
        N.gh_set_tuning(**old)
