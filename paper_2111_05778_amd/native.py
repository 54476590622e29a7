"""ctypes binding of libgh.so: the C ABI of include/gh.h, name for name.

Only argument marshalling happens here.  Device buffers are torch tensors
(passed by data_ptr) and streams are torch streams; every computation runs
in the library's HIP kernels.  Importing fails loudly when the library has
not been built: there is no fallback path.
"""
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgh.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2111_05778_amd.build`")
lib = ctypes.CDLL(_LIB_PATH)

GH_OK, GH_EINVAL, GH_ECAPACITY, GH_EHIP, GH_EUNSUPPORTED, GH_ENONFINITE = 0, -1, -2, -3, -4, -5
GH_FLAG_CAPACITY, GH_FLAG_NONFINITE, GH_FLAG_INTERNAL = 1, 2, 4
GH_SDB_PRIMS, GH_SDB_MLP = 1, 2
GH_PREC_FP32, GH_PREC_BF16, GH_PREC_BF16X3 = 0, 1, 2
GH_ACT_SOFTPLUS, GH_ACT_RELU = 0, 1
GH_BF16_HOP_FP32, GH_BF16_HOP_SHRINK = 0, 1
GH_PRIM_FLOATS = 16
GH_PRIM_TYPES = 11
GH_NOALLOC_WORKSPACE_BYTES = 128 << 20

EXPORTS = ["sdb_describe", "gh_workspace_size", "gh_hop", "gh_hop_traced", "gh_cont_workspace_size", "gh_cont", "gh_mc", "gh_polygonize_noalloc", "gh_dense", "gh_dense_signs_size", "gh_candidates",
           "gh_eval_points", "gh_bf16_margin", "gh_set_tuning", "gh_get_tuning", "gh_param_count", "gh_backward_workspace_size",
           "gh_backward", "gh_batch_buffer_size", "gh_batch_create", "gh_batch_run", "gh_batch_capture",
           "gh_batch_replay", "gh_batch_item_count", "gh_batch_destroy", "gh_last_error"]


class gh_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("lo", ctypes.c_float), ("h", ctypes.c_float)]


class gh_counters(ctypes.Structure):
    _fields_ = [("n_hop_evals", ctypes.c_int64), ("n_cand", ctypes.c_int64), ("n_corner", ctypes.c_int64),
                ("n_cells", ctypes.c_int64), ("n_vert", ctypes.c_int64), ("n_tri", ctypes.c_int64),
                ("n_reeval", ctypes.c_int64), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


COUNTER_FIELDS = [f for f, _ in gh_counters._fields_ if f != "reserved"]


class gh_sdb_spec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_prim", ctypes.c_int32), ("prims_h", ctypes.POINTER(ctypes.c_float)),
                ("n_freq", ctypes.c_int32), ("width", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("omegas_h", ctypes.POINTER(ctypes.c_float)),
                ("weights_h", ctypes.POINTER(ctypes.POINTER(ctypes.c_float))),
                ("biases_h", ctypes.POINTER(ctypes.POINTER(ctypes.c_float))),
                ("a_s", ctypes.c_float), ("r0", ctypes.c_float), ("a_n", ctypes.c_float), ("b", ctypes.c_float),
                ("bf16_margin", ctypes.c_float), ("activation", ctypes.c_int32), ("bf16_hop", ctypes.c_int32),
                ("bf16x3_margin", ctypes.c_float), ("bf16_offset", ctypes.c_float)]


class gh_tuning(ctypes.Structure):
    _fields_ = [("hop_lanes_per_ray", ctypes.c_int32), ("scan_blocks_per_cu", ctypes.c_int32),
                ("batch_rays_per_item", ctypes.c_int32), ("mlp_split", ctypes.c_int32),
                ("mc_items_per_thread", ctypes.c_int32), ("hop_step_budget", ctypes.c_int32),
                ("mlp_pool_tiles", ctypes.c_int32), ("mlp_spec_rows", ctypes.c_int32),
                ("mlp_lean", ctypes.c_int32), ("reserved", ctypes.c_int32)]


TUNING_FIELDS = ("hop_lanes_per_ray", "scan_blocks_per_cu", "batch_rays_per_item", "mlp_split", "mc_items_per_thread",
                 "hop_step_budget", "mlp_pool_tiles", "mlp_spec_rows", "mlp_lean")


class gh_sdb_desc(ctypes.Structure):
    _fields_ = [("opaque", ctypes.c_uint64 * 32)]


class gh_batch_item(ctypes.Structure):
    _fields_ = [("desc", gh_sdb_desc), ("grid", gh_grid), ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t),
                ("corner_cap", ctypes.c_int64), ("verts", ctypes.c_void_p), ("vert_edge", ctypes.c_void_p),
                ("vert_t", ctypes.c_void_p), ("vert_cap", ctypes.c_int64), ("tris", ctypes.c_void_p),
                ("tri_cap", ctypes.c_int64), ("cells", ctypes.c_void_p), ("cases", ctypes.c_void_p),
                ("cell_cap", ctypes.c_int64), ("ctr", ctypes.c_void_p)]


_vp, _i64, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
_P = ctypes.POINTER

lib.sdb_describe.argtypes = [_P(gh_sdb_spec), _vp, _sz, _P(_sz), _P(gh_sdb_desc), _vp]
lib.gh_workspace_size.argtypes = [_P(gh_grid), _i64, _P(_sz)]
lib.gh_hop.argtypes = [_P(gh_sdb_desc), _P(gh_grid), _vp, _sz, _i64, _vp, _vp]
lib.gh_hop_traced.argtypes = [_P(gh_sdb_desc), _P(gh_grid), _vp, _sz, _i64, _vp, _vp]
lib.gh_cont_workspace_size.argtypes = [_P(gh_grid), _i64, _P(_sz)]
lib.gh_cont.argtypes = [_P(gh_sdb_desc), _P(gh_grid), _vp, _sz, _i64, _vp, _sz, _i64, _vp, _i64, _vp, _P(_i64), _vp]
lib.gh_mc.argtypes = [_P(gh_sdb_desc), _P(gh_grid), _vp, _sz, _i64, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _i64,
                      _vp, _vp]
lib.gh_polygonize_noalloc.argtypes = [_P(gh_sdb_desc), _P(gh_grid), _i64, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp,
                                      _i64, _vp, _vp]
lib.gh_dense.argtypes = [_P(gh_sdb_desc), _P(gh_grid), _vp, _sz, _i64, _vp, _vp, _vp]
lib.gh_dense_signs_size.argtypes = [_P(gh_grid), _P(_sz)]
lib.gh_candidates.argtypes = [_P(gh_grid), _vp, _sz, _i64, _vp, _i64, _vp, _vp]
lib.gh_eval_points.argtypes = [_P(gh_sdb_desc), _vp, _vp, _i64, _vp]
lib.gh_bf16_margin.argtypes = [_P(gh_sdb_desc), ctypes.c_int32, _vp, _i64, ctypes.c_float, _vp, _vp, _vp, _vp]
lib.gh_param_count.argtypes = [_P(gh_sdb_desc), _P(_i64)]
lib.gh_backward_workspace_size.argtypes = [_P(gh_sdb_desc), _i64, _P(_sz)]
lib.gh_backward.argtypes = [_P(gh_sdb_desc), _P(gh_grid), _vp, _sz, _i64, _vp, _vp, _vp, _sz, _vp, _vp]
lib.gh_batch_buffer_size.argtypes = [ctypes.c_int, _P(gh_batch_item), _P(_sz)]
lib.gh_batch_create.argtypes = [ctypes.c_int, _P(gh_batch_item), _vp, _sz, _vp, _P(_vp)]
lib.gh_batch_run.argtypes = [_vp, _vp]
lib.gh_batch_capture.argtypes = [_vp, _vp]
lib.gh_batch_replay.argtypes = [_vp, _vp]
lib.gh_batch_item_count.argtypes = [_vp, _P(_i64)]
lib.gh_batch_destroy.argtypes = [_vp]
lib.gh_set_tuning.argtypes = [_P(gh_tuning)]
lib.gh_get_tuning.argtypes = [_P(gh_tuning)]
lib.gh_last_error.restype = ctypes.c_char_p
for _name in EXPORTS[:-1]:
    getattr(lib, _name).restype = ctypes.c_int


class GhError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib.gh_last_error().decode(errors="replace")
        super().__init__(f"{where} returned {status}: {msg}")


def check(status, where):
    if status != GH_OK:
        raise GhError(status, where)


def ptr(t):
    """Device pointer of a tensor, or NULL for None."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_grid(n, lo, h):
    return gh_grid(int(n), float(lo), float(h))


# ------------------------------------------------------------ thin wrappers
def sdb_describe(spec, dev_blob, blob_bytes, desc, stream=None):
    need = _sz(0)
    st = lib.sdb_describe(ctypes.byref(spec), ptr(dev_blob), blob_bytes, ctypes.byref(need),
                          ctypes.byref(desc) if desc is not None else None, stream_handle(stream))
    return st, need.value


def gh_workspace_size(grid, corner_cap=0):
    out = _sz(0)
    check(lib.gh_workspace_size(ctypes.byref(grid), int(corner_cap), ctypes.byref(out)), "gh_workspace_size")
    return out.value


def gh_hop(desc, grid, ws, corner_cap, ctr, stream=None):
    return lib.gh_hop(ctypes.byref(desc), ctypes.byref(grid), ptr(ws), ws.numel() * ws.element_size(),
                      int(corner_cap), ptr(ctr), stream_handle(stream))


def gh_hop_traced(desc, grid, ws, corner_cap, ctr, stream=None):
    return lib.gh_hop_traced(ctypes.byref(desc), ctypes.byref(grid), ptr(ws), ws.numel() * ws.element_size(),
                             int(corner_cap), ptr(ctr), stream_handle(stream))


def gh_cont_workspace_size(grid, frontier_cap=0):
    out = _sz(0)
    check(lib.gh_cont_workspace_size(ctypes.byref(grid), int(frontier_cap), ctypes.byref(out)), "gh_cont_workspace_size")
    return out.value


def gh_cont(desc, grid, ws, corner_cap, cws, frontier_cap, seeds, ctr, stream=None):
    """Returns the number of levels."""
    levels = _i64(0)
    check(lib.gh_cont(ctypes.byref(desc), ctypes.byref(grid), ptr(ws), ws.numel() * ws.element_size(), int(corner_cap),
                      ptr(cws), cws.numel() * cws.element_size(), int(frontier_cap), ptr(seeds), seeds.numel(), ptr(ctr),
                      ctypes.byref(levels), stream_handle(stream)), "gh_cont")
    return levels.value


def gh_dense(desc, grid, ws, corner_cap, signs, ctr, stream=None):
    return lib.gh_dense(ctypes.byref(desc), ctypes.byref(grid), ptr(ws), ws.numel() * ws.element_size(),
                        int(corner_cap), ptr(signs), ptr(ctr), stream_handle(stream))


def gh_dense_signs_size(grid):
    out = _sz(0)
    check(lib.gh_dense_signs_size(ctypes.byref(grid), ctypes.byref(out)), "gh_dense_signs_size")
    return out.value


def gh_mc(desc, grid, ws, corner_cap, verts, vert_edge, vert_t, vert_cap, tris, tri_cap, cells, cases, cell_cap,
          ctr, stream=None):
    return lib.gh_mc(ctypes.byref(desc), ctypes.byref(grid), ptr(ws), ws.numel() * ws.element_size(),
                     int(corner_cap), ptr(verts), ptr(vert_edge), ptr(vert_t), int(vert_cap), ptr(tris),
                     int(tri_cap), ptr(cells), ptr(cases), int(cell_cap), ptr(ctr), stream_handle(stream))


def gh_polygonize_noalloc(desc, grid, corner_cap, verts, vert_edge, vert_t, vert_cap, tris, tri_cap, cells, cases,
                          cell_cap, ctr, stream=None):
    return lib.gh_polygonize_noalloc(ctypes.byref(desc), ctypes.byref(grid), int(corner_cap), ptr(verts),
                                     ptr(vert_edge), ptr(vert_t), int(vert_cap), ptr(tris), int(tri_cap), ptr(cells),
                                     ptr(cases), int(cell_cap), ptr(ctr), stream_handle(stream))


def gh_candidates(grid, ws, corner_cap, out, cap, ctr, stream=None):
    return lib.gh_candidates(ctypes.byref(grid), ptr(ws), ws.numel() * ws.element_size(), int(corner_cap),
                             ptr(out), int(cap), ptr(ctr), stream_handle(stream))


def gh_eval_points(desc, xyz, f, m, stream=None):
    return lib.gh_eval_points(ctypes.byref(desc), ptr(xyz), ptr(f), int(m), stream_handle(stream))


def gh_bf16_margin(desc, precision, xyz, m, factor, f32, flp, margin, offset=None, stream=None):
    return lib.gh_bf16_margin(ctypes.byref(desc), int(precision), ptr(xyz), int(m), float(factor), ptr(f32), ptr(flp),
                              ptr(margin), ptr(offset), stream_handle(stream))


def gh_set_tuning(hop_lanes_per_ray=0, scan_blocks_per_cu=0, batch_rays_per_item=0, mlp_split=0,
                  mc_items_per_thread=0, hop_step_budget=0, mlp_pool_tiles=0, mlp_spec_rows=0,
                  mlp_lean=0):
    """Process-wide launch shapes; 0 keeps the built-in choice (see include/gh.h)."""
    t = gh_tuning()
    t.hop_lanes_per_ray = int(hop_lanes_per_ray)
    t.scan_blocks_per_cu = int(scan_blocks_per_cu)
    t.batch_rays_per_item = int(batch_rays_per_item)
    t.mlp_split = int(mlp_split)
    t.mc_items_per_thread = int(mc_items_per_thread)
    t.hop_step_budget = int(hop_step_budget)
    t.mlp_pool_tiles = int(mlp_pool_tiles)
    t.mlp_spec_rows = int(mlp_spec_rows)
    t.mlp_lean = int(mlp_lean)
    check(lib.gh_set_tuning(ctypes.byref(t)), "gh_set_tuning")


def gh_get_tuning():
    t = gh_tuning()
    check(lib.gh_get_tuning(ctypes.byref(t)), "gh_get_tuning")
    return {f: int(getattr(t, f)) for f in TUNING_FIELDS}


def gh_param_count(desc):
    out = _i64(0)
    check(lib.gh_param_count(ctypes.byref(desc), ctypes.byref(out)), "gh_param_count")
    return out.value


def gh_backward_workspace_size(desc, corner_cap):
    out = _sz(0)
    check(lib.gh_backward_workspace_size(ctypes.byref(desc), int(corner_cap), ctypes.byref(out)),
          "gh_backward_workspace_size")
    return out.value


def gh_backward(desc, grid, ws, corner_cap, dL_dverts, dL_dtheta, bws, ctr, stream=None):
    return lib.gh_backward(ctypes.byref(desc), ctypes.byref(grid), ptr(ws), ws.numel() * ws.element_size(),
                           int(corner_cap), ptr(dL_dverts), ptr(dL_dtheta), ptr(bws),
                           bws.numel() * bws.element_size(), ptr(ctr), stream_handle(stream))


def gh_batch_buffer_size(items):
    out = _sz(0)
    check(lib.gh_batch_buffer_size(len(items), items, ctypes.byref(out)), "gh_batch_buffer_size")
    return out.value


def gh_batch_create(items, buf, stream=None):
    handle = _vp()
    check(lib.gh_batch_create(len(items), items, ptr(buf), buf.numel(), stream_handle(stream), ctypes.byref(handle)),
          "gh_batch_create")
    return handle


def gh_batch_run(handle, stream=None):
    return lib.gh_batch_run(handle, stream_handle(stream))


def gh_batch_capture(handle, stream=None):
    return lib.gh_batch_capture(handle, stream_handle(stream))


def gh_batch_replay(handle, stream=None):
    return lib.gh_batch_replay(handle, stream_handle(stream))


def gh_batch_item_count(handle):
    out = _i64(0)
    check(lib.gh_batch_item_count(handle, ctypes.byref(out)), "gh_batch_item_count")
    return out.value


def gh_batch_destroy(handle):
    return lib.gh_batch_destroy(handle)
