"""Device buffers and call sequences around the C ABI.

`Bound` uploads a distance bound once (sdb_describe); `Polygonizer` owns the
workspace, counters and outputs for one grid and enqueues gh_hop (or
gh_dense) followed by gh_mc on a torch stream.  `run()` waits, reads the
counters, and re-runs with larger buffers when a capacity was too small.
Every step of the method runs in the library's kernels.
"""
import ctypes

import numpy as np
import torch

from . import native as N


class Bound:
    """A bound packed into a device blob; keep it alive while it is used."""

    def __init__(self, spec, keep, device):
        self.spec = spec
        self._keep = keep
        st, need = N.sdb_describe(spec, None, 0, None)
        N.check(st, "sdb_describe(size)")
        self.blob = torch.empty(max(need, 1), dtype=torch.uint8, device=device)
        self.desc = N.gh_sdb_desc()
        st, _ = N.sdb_describe(spec, self.blob, need, self.desc)
        N.check(st, "sdb_describe")

    @staticmethod
    def prims(records, device="cuda"):
        """Min-union of primitive records (n x 16 float32, see include/gh.h)."""
        rec = np.ascontiguousarray(np.asarray(records, dtype=np.float32).reshape(-1, N.GH_PRIM_FLOATS))
        spec = N.gh_sdb_spec()
        spec.kind = N.GH_SDB_PRIMS
        spec.n_prim = rec.shape[0]
        spec.prims_h = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        return Bound(spec, [rec], device)

    @staticmethod
    def mlp(net, precision="fp32", margin=None, device="cuda", hop="fp32", margin3=0.0, offset=0.0):
        """Neural bound f = a_s (||p|| - r0) + a_n NN(gamma(p)) + b.

        net: dict with "omegas" (F), "weights" (depth+1 arrays, fan_out x
        fan_in), "biases", the scalars "a_s", "r0", "a_n", "b", and
        optionally "activation" ("softplus", the default, or "relu").
        precision: "fp32", "bf16" or "bf16x3".
        margin: eps >= |f_bf16 - f_fp32|, required (> 0) for the bf16
        precisions, whose hop tests and signs it certifies: measure it with
        bf16_margin() over points covering the grid's cube.
        hop: rule of the bf16 hop, "fp32" (ambiguous steps re-evaluated in
        FP32: the FP32 schedule) or "shrink" (steps of
        floor(max(|f| - margin, 0)/h) from the bf16 value alone).
        margin3 (plain bf16 only): eps3 >= |f_bf16x3 - f_fp32|; corner values
        within margin of zero are then certified by a split-bf16 value first
        and go to FP32 only within margin3 of zero (0: FP32 directly).
        offset (plain bf16 only): subtracted from every bf16 value; measure it
        with the margin, bf16_margin(..., with_offset=True), which then
        bounds |f_bf16 - offset - f_fp32|."""
        if precision != "fp32" and margin is None:
            raise ValueError(f"precision {precision!r} needs a margin: pass margin=bf16_margin(net, points, "
                             f"{precision!r}) with points covering the grid's cube")
        ws = [np.ascontiguousarray(np.asarray(w, dtype=np.float32)) for w in net["weights"]]
        bs = [np.ascontiguousarray(np.asarray(b, dtype=np.float32)) for b in net["biases"]]
        om = np.ascontiguousarray(np.asarray(net["omegas"], dtype=np.float32))
        fp = ctypes.POINTER(ctypes.c_float)
        wptr = (fp * len(ws))(*[w.ctypes.data_as(fp) for w in ws])
        bptr = (fp * len(bs))(*[b.ctypes.data_as(fp) for b in bs])
        spec = N.gh_sdb_spec()
        spec.kind = N.GH_SDB_MLP
        spec.n_freq = len(om)
        spec.width = ws[0].shape[0]
        spec.depth = len(ws) - 1
        spec.precision = {"fp32": N.GH_PREC_FP32, "bf16": N.GH_PREC_BF16, "bf16x3": N.GH_PREC_BF16X3}[precision]
        spec.activation = {"softplus": N.GH_ACT_SOFTPLUS, "relu": N.GH_ACT_RELU}[net.get("activation", "softplus")]
        spec.omegas_h = om.ctypes.data_as(fp)
        spec.weights_h = wptr
        spec.biases_h = bptr
        spec.a_s, spec.r0, spec.a_n, spec.b = (float(net[k]) for k in ("a_s", "r0", "a_n", "b"))
        spec.bf16_margin = float(margin or 0.0)
        spec.bf16_hop = {"fp32": N.GH_BF16_HOP_FP32, "shrink": N.GH_BF16_HOP_SHRINK}[hop]
        spec.bf16x3_margin = float(margin3)
        spec.bf16_offset = float(offset)
        return Bound(spec, [ws, bs, om, wptr, bptr], device)

    def eval(self, xyz):
        """Bound values at points (m x 3 float32 device tensor)."""
        xyz = xyz.contiguous()
        f = torch.empty(xyz.shape[0], dtype=torch.float32, device=xyz.device)
        N.check(N.gh_eval_points(self.desc, xyz, f, xyz.shape[0]), "gh_eval_points")
        return f


def bf16_margin(net, points, precision="bf16", factor=2.0, device="cuda", with_offset=False):
    """Margin of the bf16 decisions: factor * max |f_bf16 - f_fp32| over the
    given points, computed by gh_bf16_margin with the library's own
    evaluators (one call; the result is read back).  with_offset: returns
    (margin, offset), offset the midrange of f_bf16 - f_fp32 and margin
    factor times half its range, to pass as Bound.mlp(margin=, offset=)."""
    pts = torch.as_tensor(np.asarray(points, dtype=np.float32), device=device).reshape(-1, 3).contiguous()
    m = pts.shape[0]
    bound = Bound.mlp(net, "fp32", device=device)
    f32 = torch.empty(max(m, 1), dtype=torch.float32, device=device)
    flp = torch.empty(max(m, 1), dtype=torch.float32, device=device)
    out = torch.empty(2, dtype=torch.float32, device=device)
    prec = {"bf16": N.GH_PREC_BF16, "bf16x3": N.GH_PREC_BF16X3}[precision]
    N.check(N.gh_bf16_margin(bound.desc, prec, pts, m, factor, f32, flp, out[0:1], out[1:2] if with_offset else None),
            "gh_bf16_margin")
    if with_offset:
        margin, offset = out.tolist()
        return margin, offset
    return float(out[0].item())


def counters_dict(ctr):
    v = ctr.cpu().numpy()
    out = {name: int(v[q]) for q, name in enumerate(N.COUNTER_FIELDS[:-1])}
    out["flags"] = int(v[7]) & 0xFFFFFFFF
    return out


class Mesh:
    def __init__(self, verts, vert_edge, vert_t, tris, cells, cases, counters):
        self.verts, self.vert_edge, self.vert_t = verts, vert_edge, vert_t
        self.tris, self.cells, self.cases = tris, cells, cases
        self.counters = counters


class Polygonizer:
    """Buffers and call sequence for one bound on one grid (n, lo, h)."""

    def __init__(self, bound, n, lo, h, corner_cap=0, vert_cap=0, tri_cap=0, cell_cap=0, device="cuda",
                 keep_cells=True, keep_edges=True, tuning=None):
        """tuning: launch shapes applied (process-wide) before each enqueue: a
        dict of gh_tuning fields, "auto" for the autotuner's cached choice for
        this workload (defaults when none is cached), or None to leave the
        current setting alone."""
        self.bound = bound
        self.grid = N.make_grid(n, lo, h)
        self.n = int(n)
        self.device = torch.device(device)
        n1 = self.n + 1
        self.corner_cap = int(corner_cap) if corner_cap > 0 else 16 * n1 * n1
        self.vert_cap = int(vert_cap) if vert_cap > 0 else 8 * n1 * n1
        self.tri_cap = int(tri_cap) if tri_cap > 0 else 2 * self.vert_cap
        self.cell_cap = int(cell_cap) if cell_cap > 0 else self.tri_cap
        self.keep_cells, self.keep_edges = keep_cells, keep_edges
        self.ctr = torch.zeros(8, dtype=torch.int64, device=self.device)
        self.dense_buf = None
        self._cws = None
        if tuning == "auto":
            from . import autotune
            tuning = autotune.lookup(autotune.signature(bound.spec, self.n), self.device) or {}
        self.tuning = tuning
        self._alloc()

    @property
    def tuning(self):
        return self._tuning

    @tuning.setter
    def tuning(self, t):
        """Launch shapes (dict of gh_tuning fields; missing or zero fields keep
        the built-in choice), applied before each enqueue; None leaves the
        process-wide setting alone."""
        self._tuning = None if t is None else dict(t)
        self._tuning_struct = None
        if t is not None:
            st = N.gh_tuning()
            for f in N.TUNING_FIELDS:
                setattr(st, f, int(t.get(f, 0)))
            self._tuning_struct = st

    def _alloc(self):
        dev = self.device
        ws_bytes = N.gh_workspace_size(self.grid, self.corner_cap)
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        self.verts = torch.empty((self.vert_cap, 3), dtype=torch.float32, device=dev)
        self.vert_edge = torch.empty(self.vert_cap, dtype=torch.int64, device=dev) if self.keep_edges else None
        self.vert_t = torch.empty(self.vert_cap, dtype=torch.float32, device=dev) if self.keep_edges else None
        self.tris = torch.empty((self.tri_cap, 3), dtype=torch.int32, device=dev)
        self.cells = torch.empty(self.cell_cap, dtype=torch.int64, device=dev) if self.keep_cells else None
        self.cases = torch.empty(self.cell_cap, dtype=torch.uint8, device=dev) if self.keep_cells else None

    # ---------------------------------------------------------- enqueue only
    def _apply_tuning(self):
        if self._tuning_struct is not None:  # one host call: the enqueue path stays lean
            N.check(N.lib.gh_set_tuning(ctypes.byref(self._tuning_struct)), "gh_set_tuning")

    def enqueue_hop(self, stream=None):
        self._apply_tuning()
        N.check(N.gh_hop(self.bound.desc, self.grid, self.ws, self.corner_cap, self.ctr, stream), "gh_hop")

    def enqueue_hop_traced(self, stream=None):
        """The paper's per-column procedure taken literally (gh_hop_traced);
        analytic bounds only."""
        self._apply_tuning()
        N.check(N.gh_hop_traced(self.bound.desc, self.grid, self.ws, self.corner_cap, self.ctr, stream),
                "gh_hop_traced")

    def enqueue_cont(self, seeds, frontier_cap=0, stream=None):
        """Continuation (gh_cont) from seed cells, an int64 device tensor of
        cell ids; analytic bounds only.  Blocks until the search is done and
        returns its number of levels."""
        self._apply_tuning()
        nb = N.gh_cont_workspace_size(self.grid, frontier_cap)
        if self._cws is None or self._cws.numel() < nb:
            self._cws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        return N.gh_cont(self.bound.desc, self.grid, self.ws, self.corner_cap, self._cws, frontier_cap, seeds,
                         self.ctr, stream)

    def enqueue_dense(self, stream=None):
        self._apply_tuning()
        if self.dense_buf is None:
            nb = N.gh_dense_signs_size(self.grid)
            self.dense_buf = torch.empty(nb // 4, dtype=torch.int32, device=self.device)
        N.check(N.gh_dense(self.bound.desc, self.grid, self.ws, self.corner_cap, self.dense_buf, self.ctr, stream),
                "gh_dense")

    def enqueue_mc(self, stream=None):
        self._apply_tuning()
        N.check(N.gh_mc(self.bound.desc, self.grid, self.ws, self.corner_cap, self.verts, self.vert_edge,
                        self.vert_t, self.vert_cap, self.tris, self.tri_cap, self.cells, self.cases,
                        self.cell_cap if self.keep_cells else 0, self.ctr, stream), "gh_mc")

    # ------------------------------------------------------------ graphs
    def capture(self, dense=False):
        """Records one hop (or enumeration) and marching cubes into a graph;
        replay() launches it again with no per-kernel host work.  The buffers
        must already be large enough (run() once first): a replay does not
        grow them, and the counters report any shortfall as after run()."""
        self._graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.graph(self._graph, stream=side):
            (self.enqueue_dense if dense else self.enqueue_hop)()
            self.enqueue_mc()
        torch.cuda.current_stream(self.device).wait_stream(side)

    def replay(self):
        self._graph.replay()

    # ------------------------------------------------------------ blocking
    def run(self, dense=False, stream=None, max_retries=3, traced=False, seeds=None):
        """Cells by grid hopping (or enumeration with dense, the literal
        traced procedure with traced, or continuation from the given seed
        cells), then marching cubes; blocks."""
        first = self.enqueue_dense if dense else (self.enqueue_hop_traced if traced else self.enqueue_hop)
        if seeds is not None:
            first = lambda st: self.enqueue_cont(seeds, stream=st)  # noqa: E731
        for _ in range(max_retries + 1):
            first(stream)
            self.enqueue_mc(stream)
            torch.cuda.synchronize(self.device)
            c = counters_dict(self.ctr)
            if c["flags"] & N.GH_FLAG_INTERNAL:
                raise RuntimeError("inconsistent workspace contents or an unbounded trace (library bug)")
            if c["flags"] & N.GH_FLAG_NONFINITE:
                raise FloatingPointError("the bound returned a non-finite value")
            if not c["flags"] & N.GH_FLAG_CAPACITY:
                return self.result(c)
            self.corner_cap = max(self.corner_cap, int(c["n_corner"] * 1.25) + 64)
            self.vert_cap = max(self.vert_cap, int(c["n_vert"] * 1.25) + 64)
            self.tri_cap = max(self.tri_cap, int(c["n_tri"] * 1.25) + 64)
            self.cell_cap = max(self.cell_cap, int(c["n_cells"] * 1.25) + 64)
            self._alloc()
        raise RuntimeError("capacity retries exhausted")

    def result(self, c=None):
        c = c or counters_dict(self.ctr)
        nv, nt, nc = c["n_vert"], c["n_tri"], c["n_cells"]
        return Mesh(self.verts[:nv], self.vert_edge[:nv] if self.keep_edges else None,
                    self.vert_t[:nv] if self.keep_edges else None, self.tris[:nt],
                    self.cells[:nc] if self.keep_cells else None, self.cases[:nc] if self.keep_cells else None, c)

    def candidates(self, stream=None):
        """Candidate cell ids recorded by the last hop (ascending int64)."""
        c = counters_dict(self.ctr)
        out = torch.empty(max(c["n_cand"], 1), dtype=torch.int64, device=self.device)
        N.check(N.gh_candidates(self.grid, self.ws, self.corner_cap, out, c["n_cand"], self.ctr, stream),
                "gh_candidates")
        torch.cuda.synchronize(self.device)
        return out[:c["n_cand"]]


class BatchPolygonizer:
    """Many (bound, grid) pairs through gh_batch_*: one persistent hop launch,
    marching cubes per shape, optionally replayed from a captured hipGraph.

    shapes: list of (Bound, n, lo, h).  Buffers are sized like Polygonizer's
    defaults; run() re-plans with larger buffers when a capacity was short."""

    def __init__(self, shapes, device="cuda", keep_cells=True):
        self.device = torch.device(device)
        self.polys = [Polygonizer(b, n, lo, h, device=self.device, keep_cells=keep_cells) for (b, n, lo, h) in shapes]
        self._plan()

    def _plan(self):
        self.items = (N.gh_batch_item * len(self.polys))()
        for it, p in zip(self.items, self.polys):
            it.desc = p.bound.desc
            it.grid = p.grid
            it.ws, it.ws_bytes, it.corner_cap = p.ws.data_ptr(), p.ws.numel(), p.corner_cap
            it.verts, it.vert_cap = p.verts.data_ptr(), p.vert_cap
            it.vert_edge = p.vert_edge.data_ptr() if p.vert_edge is not None else None
            it.vert_t = p.vert_t.data_ptr() if p.vert_t is not None else None
            it.tris, it.tri_cap = p.tris.data_ptr(), p.tri_cap
            it.cells = p.cells.data_ptr() if p.cells is not None else None
            it.cases = p.cases.data_ptr() if p.cases is not None else None
            it.cell_cap = p.cell_cap if p.keep_cells else 0
            it.ctr = p.ctr.data_ptr()
        self.buf = torch.empty(N.gh_batch_buffer_size(self.items), dtype=torch.uint8, device=self.device)
        self.handle = N.gh_batch_create(self.items, self.buf)
        self.captured = False

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            N.gh_batch_destroy(h)

    def item_count(self):
        return N.gh_batch_item_count(self.handle)

    def enqueue(self, stream=None):
        N.check(N.gh_batch_run(self.handle, stream), "gh_batch_run")

    def capture(self):
        """Records the batch into a hipGraph.  Capture needs a stream other
        than the null stream, so the graph lives on a side stream that
        replay() orders after, and before, torch's current stream."""
        self.graph_stream = torch.cuda.Stream(self.device)
        self.graph_stream.wait_stream(torch.cuda.current_stream(self.device))
        N.check(N.gh_batch_capture(self.handle, self.graph_stream), "gh_batch_capture")
        self.captured = True

    def replay(self):
        cur = torch.cuda.current_stream(self.device)
        self.graph_stream.wait_stream(cur)
        N.check(N.gh_batch_replay(self.handle, self.graph_stream), "gh_batch_replay")
        cur.wait_stream(self.graph_stream)

    def run(self, max_retries=3):
        for _ in range(max_retries + 1):
            self.enqueue()
            torch.cuda.synchronize(self.device)
            cs = [counters_dict(p.ctr) for p in self.polys]
            if any(c["flags"] & (N.GH_FLAG_INTERNAL | N.GH_FLAG_NONFINITE) for c in cs):
                raise RuntimeError(f"batch flags: {[c['flags'] for c in cs]}")
            short = [c["flags"] & N.GH_FLAG_CAPACITY for c in cs]
            if not any(short):
                return [p.result(c) for p, c in zip(self.polys, cs)]
            for p, c, sh in zip(self.polys, cs, short):
                if sh:
                    p.corner_cap = max(p.corner_cap, int(c["n_corner"] * 1.25) + 64)
                    p.vert_cap = max(p.vert_cap, int(c["n_vert"] * 1.25) + 64)
                    p.tri_cap = max(p.tri_cap, int(c["n_tri"] * 1.25) + 64)
                    p.cell_cap = max(p.cell_cap, int(c["n_cells"] * 1.25) + 64)
                    p._alloc()
            N.gh_batch_destroy(self.handle)
            self.handle = None
            self._plan()
        raise RuntimeError("capacity retries exhausted")

    def results(self):
        return [p.result() for p in self.polys]
