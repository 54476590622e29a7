"""Benchmark: grid cells polygonized per second (N^3 / t) by grid hopping.

One step = gh_hop + gh_mc over the whole grid (hop over all N^2 ray columns,
distinct corner evaluation, welded vertex and triangle emit) with every
input already resident in HBM.  Workload: min-union of 12 seeded
primitives (sphere, box, torus, capsule; seed 0) on [-1, 1]^3 at N = 512,
float32.  The enumeration path (bound at all (N+1)^3 lattice points,
marching cubes on every cell, same emit) is timed beside it.  Both are timed
as replays of a captured graph of the step (ms_per_step, value); the eager
per-call launches are timed too (ms_per_step_eager) and give the per-phase
split (roofline.hop_ms, mc_ms).

Prints one JSON line.  Extra objects:
  roofline      the hop kernel against the FP32 peak of the chip (157.3 TFLOP/s),
                and against the issue ceiling of its unfused FP32 operations
  cpu_baseline  the oracle (FP64 numpy) on the same workload on all host cores
                (at most 16), with the one-thread time beside it
  neural        the network bound (width 256, depth 4, 16 frequencies) at
                N = 512 in bf16 on MFMA with FP32 accumulation: the hop steps
                shortened by the bf16 margin (no FP32 in the hop), corner
                signs certified by split bf16 and FP32; its MFMA roofline and
                the enumeration path (same certification) beside it
  neural_bf16x3 the same network in split bf16 (hi*hi + hi*lo + lo*hi) with
                the FP32 hop schedule, its roofline and its enumeration
  paper_net     the same for the paper's network shape (eight ReLU layers of
                width 64 on raw coordinates, random weights): the
                small-width MFMA regime
  backward      the adjoint of the mean squared vertex-to-target loss for the
                same network at N = 256, FP32 forward (milliseconds)
  batch         64 bounds on grids of 64..512, one persistent hop launch plus
                marching cubes per shape, replayed from a hipGraph
  cont          continuation (gh_cont, the paper's surface-following
                comparator) on the headline workload from one seed per
                surface component, with marching cubes
  primitives    the paper's first scene's seven primitive types (sphere,
                cube, cone, cylinder, torus, hexagonal prism, capsule) at
                N = 512, with the enumeration path beside it
  traced        the paper's per-column procedure taken literally
                (gh_hop_traced: sphere tracing to sqrt(6)/2 h) on the headline
                workload, with marching cubes on its candidates, its counts,
                and the number of sign-change cells it leaves out
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (dense, no sparsity).
PEAK_FP32 = 157.3e12        # FP32 vector: an FMA counts two FLOP, packed dual-FP32 two more
PEAK_FP32_MFMA = 157.3e12   # FP32 on the matrix cores
PEAK_BF16_MFMA = 2.5e15
HBM_PEAK = 8.0e12
# Issue ceiling of the analytic bounds' arithmetic: 256 CUs x 64 lanes x 2.4 GHz
# = 39.3e12 FP32 operations/s, one operation per lane per clock.  Their
# formulas can use neither the FMA (contraction is off: each operation is
# rounded on its own) nor packed dual-FP32 (disabled on this target), so
# this is the most they can reach; it is reported beside the published peak.
PEAK_FP32_ISSUE = 256 * 64 * 2.4e9

# FP32 operations per evaluation of each primitive type, counted from the
# formula in include/gh.h.  Counting rule: every add, sub, mul, min, max, abs,
# neg, compare, select and square root of the formula is one operation (the
# square root one, though the hardware takes several instructions for a
# correctly rounded one); loads, the loop and the hop's own control are not
# counted.  These are the FLOP of the analytic rooflines:
# translate 3 + rotate 15 = 18 shared, then
#   sphere  3 mul + 2 add + sqrt + sub                          = 7
#   box     3 abs + 3 sub + 2 max + 3 max + 3 mul + 2 add + sqrt + min + add = 19
#   torus   2 mul + add + sqrt + sub, 2 mul + add + sqrt + sub  = 10
#   capsule neg + max + min + sub + 3 mul + 2 add + sqrt + sub = 11
#   plane   3 mul + 2 add + sub (no translate/rotate)          = 6 total
#   boxbound 3 abs + 3 sub + 2 max                              = 8
#   cylinder 2 mul + add + sqrt, sub, abs + sub, 2 max, 2 mul + add + sqrt,
#            max + min + add                                    = 16
#   cone     2 mul + add + sqrt, mul + sub + mul + sub, abs + sub + max = 11
#   hexprism 2 mul, abs + sub, add + abs + sub, sub + abs + sub, abs + sub,
#            3 max                                              = 15
#   genus2   3 mul (squares), sub, add, mul + mul + sub + mul + mul, mul + add,
#            mul + sub + mul + sub, mul (k)                        = 18
#   sierpinski per level: add + sub (u, w), 4 add/sub (e), 3 compares, 4
#            selects, 3 mul + 3 sub (q = 2q - v), mul (v_z) = 20; at the end
#            20 as per level (e, nearest vertex), 7 min/max, 2 sub, 5 for the
#            two region tests, the three distances (mul; 6 + sqrt; 5 + sqrt),
#            2 selects, ldexp, mul (k) = 52: 52 + 20 d
OPS = {0: 18 + 7, 1: 18 + 19, 2: 18 + 10, 3: 18 + 11, 4: 6, 5: 18 + 8, 6: 18 + 16, 7: 18 + 11, 8: 18 + 15,
       9: 18 + 18}


def prim_ops(r):
    t = int(r[0])
    return 18 + 52 + 20 * int(r[14]) if t == 10 else OPS[t]


def ops_per_eval(records):
    return sum(prim_ops(r) for r in records) + (len(records) - 1)   # plus the union minima


def mlp_flop_per_point(width, depth, n_freq):
    """Multiply-adds x 2 of one network evaluation (features, hidden layers, output)."""
    k1 = 3 + 6 * n_freq
    return 2 * (k1 * width + (depth - 1) * width * width + width)


def vjp_flop_per_corner(width, depth, n_freq):
    """Multiply-adds x 2 of the adjoint at one corner: the forward products
    again, the weight-gradient products of every layer (the same count), and
    the products that carry dL/dz back through the hidden layers."""
    return 2 * mlp_flop_per_point(width, depth, n_freq) + 2 * (depth - 1) * width * width


# Sources each profiled kernel is built from; a committed traffic figure is
# used only while these files are unchanged.
KERNEL_SOURCES = {
    "k_hop": ("gh_kernels.hip", "gh_device.h", "gh_hop.h"),
    "k_hop_mlp": ("gh_mlp.hip", "gh_mlp.h", "gh_hop.h", "gh_device.h"),
}


def kernel_source_hash(kernel):
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2111_05778_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel
    calibration) from the committed PMC summary, if it was taken on the
    current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    e = t.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash(kernel):
        return None
    return e["bytes_per_launch"]


def _oracle_hop_band(args):
    """One worker of the all-cores leg: the oracle's hop over a band of columns."""
    from threadpoolctl import threadpool_limits

    from oracle import hop as ohop
    from oracle import sdb as osdb
    recs, n, lo, h, columns = args
    with threadpool_limits(1):
        cells, evals, col_evals = ohop.hop(osdb.SDB.prims(recs), n, lo, h, columns=columns)
    return cells, evals, col_evals


def cpu_baseline(recs, n, lo, h):
    """The oracle as it stands (FP64 grid hopping + marching cubes) on the
    host, timed twice: one thread, and all the host cores this process may
    use (at most 16), where a pool of forked workers runs the oracle's hop on
    bands of columns (columns are independent) and marching cubes follow on
    the union of their cells.  Runs before anything touches the GPU (the
    workers are forked)."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import hop as ohop
    from oracle import sdb as osdb
    S = osdb.SDB.prims(recs)
    times = []
    with threadpool_limits(1):
        for _ in range(2):
            t0 = time.perf_counter()
            ohop.gridhop(S, n, lo, h)
            times.append(time.perf_counter() - t0)
    t1 = min(times)
    host = len(os.sched_getaffinity(0))
    cores = max(1, min(16, host))
    bands = np.array_split(np.arange(n * n, dtype=np.int64), cores * 4)
    times = []
    with mp.get_context("fork").Pool(cores) as pool:
        for _ in range(2):
            t0 = time.perf_counter()
            parts = pool.map(_oracle_hop_band, [(recs, n, lo, h, b) for b in bands])
            cells = np.sort(np.concatenate([p[0] for p in parts]))
            with threadpool_limits(1):
                ohop.polygonize_cells(S, n, lo, h, cells, sum(p[1] for p in parts),
                                      np.concatenate([p[2] for p in parts]))
            times.append(time.perf_counter() - t0)
    tc = min(times)
    return {"value": n ** 3 / tc, "unit": "cells/s", "cores": cores, "kind": "oracle",
            "sample": f"the full workload (N={n}, all {n * n} columns), best of 2 runs, {tc:.2f} s: the hop on "
                      f"{len(bands)} column bands over {cores} forked workers (host affinity {host} CPUs), "
                      f"marching cubes on one",
            "one_thread": {"value": n ** 3 / t1, "unit": "cells/s", "cores": 1,
                           "sample": f"the full workload, best of 2 runs, {t1:.2f} s"}}


def event_ms(stream, fn, reps):
    """Mean duration (ms) of fn's enqueued work over reps runs, by HIP events
    on the stream it enqueues on."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / reps


def neural_section(dev, steps, warmup, n=512, width=256, precision="bf16", dense=True, tune=True, paper=False,
                   hop="shrink"):
    """The network bound at N = 512: the calibrated random network of width
    256 (softplus, 16 frequencies), or with paper=True the paper's shape
    (eight ReLU layers of width 64 on raw coordinates).  hop: the bf16 hop
    rule, "fp32" (ambiguous steps re-evaluated in FP32) or "shrink" (steps
    shortened by the margin, no FP32 in the hop)."""
    import torch

    import workloads as W
    from paper_2111_05778_amd.polygonize import Bound, Polygonizer, bf16_margin
    if paper:
        net, width, depth, n_freq = W.paper_net_scene(), 64, 8, 0
        workload = f"mlp_w64_d8_f0_relu_seed0_n{n}"
    else:
        net, depth, n_freq = W.neural_scene(0, width), 4, 16
        workload = f"mlp_w{width}_d4_f16_seed0_n{n}"
    n, lo, h = W.grid(n)
    probe = W.probe_points(seed=3, n=65536)
    # plain bf16: the measured offset of its error is removed (a smaller
    # margin), and corner values near zero are certified by the split form first
    offset = 0.0
    if precision == "bf16":
        margin, offset = bf16_margin(net, probe, precision, with_offset=True)
    else:
        margin = bf16_margin(net, probe, precision) if precision != "fp32" else 0.0
    margin3 = bf16_margin(net, probe, "bf16x3") if precision == "bf16" else 0.0
    poly = Polygonizer(Bound.mlp(net, precision, margin=margin if precision != "fp32" else None, device=dev, hop=hop,
                                 margin3=margin3, offset=offset), n, lo, h, device=dev, keep_cells=False)
    c0 = dict(poly.run().counters)
    tuning = None
    if tune:
        from paper_2111_05778_amd import autotune
        tuning, _, _ = autotune.tune(poly, reps=2, store=False)
        poly.tuning = tuning
    stream = torch.cuda.current_stream(dev)
    for _ in range(warmup):
        poly.enqueue_hop()
        poly.enqueue_mc()
    hop_ms = event_ms(stream, poly.enqueue_hop, steps)
    mc_ms = event_ms(stream, poly.enqueue_mc, steps)
    fpp = mlp_flop_per_point(width, depth, n_freq)
    flop = c0["n_hop_evals"] * fpp
    out = {"workload": workload, "precision": precision, "hop_rule": hop, "margin": margin, "margin3": margin3,
           "offset": offset, "tuning": tuning,
           "value": n ** 3 / ((hop_ms + mc_ms) * 1e-3), "unit": "cells/s", "hop_ms": hop_ms, "mc_ms": mc_ms,
           "counters": {k: c0[k] for k in ("n_hop_evals", "n_cand", "n_reeval", "n_corner", "n_vert", "n_tri")},
           "roofline": {"bound": "mfma", "kernel": "k_hop_mlp", "achieved": flop / (hop_ms * 1e-3) / 1e12,
                        "peak": PEAK_BF16_MFMA / 1e12, "unit": "TFLOP/s",
                        "frac": flop / (hop_ms * 1e-3) / PEAK_BF16_MFMA,
                        "traffic": load_traffic("k_hop_mlp") if (not paper and precision == "bf16"
                                                                 and hop == "shrink") else None,
                        "flop_per_point": fpp, "per_launch_flop": flop}}
    if dense:
        poly.enqueue_dense()
        poly.enqueue_mc()
        torch.cuda.synchronize(dev)
        d_ms = event_ms(stream, lambda: (poly.enqueue_dense(), poly.enqueue_mc()), 1)
        out["dense_ms"] = d_ms
        out["speedup_vs_dense"] = d_ms / (hop_ms + mc_ms)
    return out


def backward_section(dev, steps, warmup, n=256, width=256):
    import numpy as np
    import torch

    import workloads as W
    from paper_2111_05778_amd import native as N
    from paper_2111_05778_amd.polygonize import Bound, Polygonizer
    net = W.neural_scene(0, width)
    n, lo, h = W.grid(n)
    poly = Polygonizer(Bound.mlp(net, "fp32", device=dev), n, lo, h, device=dev)
    mesh = poly.run()
    V = mesh.verts
    Q = torch.tensor(W.loss_targets().astype(np.float32), device=dev)
    nearest = torch.cdist(V, Q).argmin(dim=1)
    dV = (2.0 / V.shape[0]) * (V - Q[nearest])
    desc = poly.bound.desc
    P = N.gh_param_count(desc)
    grad = torch.empty(P, dtype=torch.float32, device=dev)
    bws = torch.empty(N.gh_backward_workspace_size(desc, poly.corner_cap), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)

    def bwd():
        N.check(N.gh_backward(desc, poly.grid, poly.ws, poly.corner_cap, dV, grad, bws, poly.ctr), "gh_backward")

    for _ in range(warmup):
        bwd()
    fwd_ms = event_ms(stream, lambda: (poly.enqueue_hop(), poly.enqueue_mc()), steps)
    bwd()
    bwd_ms = event_ms(stream, bwd, steps)
    # corners the loss depends on: the distinct ends of the crossing edges
    e = mesh.vert_edge
    axis, lower = e % 3, e // 3
    n1 = n + 1
    upper = lower + torch.where(axis == 0, n1 * n1, torch.where(axis == 1, n1, 1))
    corners = int(torch.unique(torch.cat([lower, upper])).numel())
    fpc = vjp_flop_per_corner(width, 4, 16)
    flop = corners * fpc
    return {"workload": f"mlp_w{width}_d4_f16_seed0_n{n}_fp32", "backward_ms": bwd_ms, "forward_ms": fwd_ms,
            "n_vert": int(V.shape[0]), "params": P, "grad_norm": float(grad.norm()),
            "roofline": {"bound": "mfma", "kernel": "k_mlp_vjp (whole gh_backward call timed)",
                         "achieved": flop / (bwd_ms * 1e-3) / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                         "unit": "TFLOP/s", "frac": flop / (bwd_ms * 1e-3) / PEAK_FP32_MFMA, "traffic": None,
                         "corners": corners, "flop_per_corner": fpc, "per_launch_flop": flop}}


def batch_section(dev, steps, warmup, precision="bf16", tune=True):
    import torch

    import workloads as W
    from paper_2111_05778_amd.polygonize import BatchPolygonizer, Bound, bf16_margin
    scenes = W.batch_scenes()
    probe = W.probe_points(seed=3, n=65536)
    shapes = []
    for sc in scenes:
        n, lo, h = W.grid(sc["n"])
        if sc["kind"] == "csg":
            b = Bound.prims(W.csg_scene(sc["seed"], sc["n_prim"]), dev)
        else:
            net = W.neural_scene(sc["seed"], sc["width"])
            plain = precision == "bf16"   # shrunk hop, offset removed, two-step corner certification
            margin, offset = (bf16_margin(net, probe, precision, with_offset=True) if plain
                              else (bf16_margin(net, probe, precision), 0.0))
            b = Bound.mlp(net, precision, margin=margin, device=dev, hop="shrink" if plain else "fp32",
                          margin3=bf16_margin(net, probe, "bf16x3") if plain else 0.0, offset=offset)
        shapes.append((b, n, lo, h))
    tuning = None
    if tune:
        from paper_2111_05778_amd import autotune
        tuning, _, _ = autotune.tune_batch(lambda: BatchPolygonizer(shapes, device=dev, keep_cells=False),
                                           [(b, n) for (b, n, _, _) in shapes], reps=1, store=False)
        autotune.apply(tuning)             # the item size is read when the batch is planned
    batch = BatchPolygonizer(shapes, device=dev, keep_cells=False)
    res = batch.run()
    ref = [dict(m.counters) for m in res]
    batch.capture()
    for _ in range(warmup):
        batch.replay()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.replay()
    torch.cuda.synchronize(dev)
    ms = (time.perf_counter() - t0) / steps * 1e3
    from paper_2111_05778_amd.polygonize import counters_dict
    for p, c in zip(batch.polys, ref):
        assert counters_dict(p.ctr)["n_tri"] == c["n_tri"]
    # the same shapes one by one, each replaying its own captured graph (hop +
    # marching cubes), back to back on one stream
    for p in batch.polys:
        p.capture()
    for _ in range(warmup):
        for p in batch.polys:
            p.replay()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(steps):
        for p in batch.polys:
            p.replay()
    torch.cuda.synchronize(dev)
    singles_ms = (time.perf_counter() - t0) / steps * 1e3
    for p, c in zip(batch.polys, ref):
        assert counters_dict(p.ctr)["n_tri"] == c["n_tri"]
    cells = sum(sc["n"] ** 3 for sc in scenes)
    # algorithmic work of the batch's hops, per kind
    net_flop = sum(c["n_hop_evals"] * mlp_flop_per_point(sc["width"], 4, 16)
                   for sc, c in zip(scenes, ref) if sc["kind"] == "mlp")
    prim_ops = sum(c["n_hop_evals"] * ops_per_eval(W.csg_scene(sc["seed"], sc["n_prim"]))
                   for sc, c in zip(scenes, ref) if sc["kind"] == "csg")
    return {"workload": "batch64_seed2", "precision": precision, "tuning": tuning, "shapes": len(scenes), "cells": cells,
            "work_items": batch.item_count(), "ms_per_step": ms, "value": cells / (ms * 1e-3), "unit": "cells/s",
            "n_tri": sum(c["n_tri"] for c in ref),
            "singles_ms": singles_ms, "batch_over_singles": ms / singles_ms,
            "hop_evals": {"network": sum(c["n_hop_evals"] for sc, c in zip(scenes, ref) if sc["kind"] == "mlp"),
                          "analytic": sum(c["n_hop_evals"] for sc, c in zip(scenes, ref) if sc["kind"] == "csg")},
            "network_flop": net_flop, "analytic_flop": prim_ops,
            "network_tflops_over_step": net_flop / (ms * 1e-3) / 1e12}


def primitives_section(dev, steps, warmup, n=512, seed=0):
    """The paper's first scene's seven primitives (sphere, cube, cone,
    cylinder, torus, hexagonal prism, capsule) at N = 512: grid hopping and
    enumeration, each followed by marching cubes."""
    import torch

    import workloads as W
    from paper_2111_05778_amd.polygonize import Bound, Polygonizer, counters_dict
    recs = W.primitives_scene(seed)
    n, lo, h = W.grid(n)
    poly = Polygonizer(Bound.prims(recs, dev), n, lo, h, device=dev, keep_cells=False)
    poly.run()
    for _ in range(warmup):
        poly.enqueue_hop()
        poly.enqueue_mc()
    stream = torch.cuda.current_stream(dev)
    hop_ms = event_ms(stream, poly.enqueue_hop, steps)
    mc_ms = event_ms(stream, poly.enqueue_mc, steps)
    c = counters_dict(poly.ctr)
    dense_ms = event_ms(stream, lambda: (poly.enqueue_dense(), poly.enqueue_mc()), max(1, steps // 2))
    return {"workload": f"primitives7_seed{seed}_n{n}", "hop_ms": hop_ms, "mc_ms": mc_ms,
            "ms_per_step": hop_ms + mc_ms, "value": n ** 3 / ((hop_ms + mc_ms) * 1e-3), "unit": "cells/s",
            "dense_ms": dense_ms, "speedup_vs_dense": dense_ms / (hop_ms + mc_ms),
            "counters": {k: c[k] for k in ("n_hop_evals", "n_cand", "n_corner", "n_vert", "n_tri")},
            "ops_per_eval": ops_per_eval(recs)}


def sierpinski_section(dev, steps, warmup, n=512, depth=8):
    """The Sierpinski tetrahedron (Section 5.1's fractal scene) at N = 512,
    depth 8 (65,536 tetrahedra of about 2.4 cells per edge): grid hopping
    and enumeration, each followed by marching cubes."""
    import torch

    import workloads as W
    from paper_2111_05778_amd.polygonize import Bound, Polygonizer, counters_dict
    recs = W.sierpinski_scene(depth)
    n, lo, h = W.grid(n)
    poly = Polygonizer(Bound.prims(recs, dev), n, lo, h, device=dev, keep_cells=False)
    poly.run()
    for _ in range(warmup):
        poly.enqueue_hop()
        poly.enqueue_mc()
    stream = torch.cuda.current_stream(dev)
    hop_ms = event_ms(stream, poly.enqueue_hop, steps)
    mc_ms = event_ms(stream, poly.enqueue_mc, steps)
    c = counters_dict(poly.ctr)
    dense_ms = event_ms(stream, lambda: (poly.enqueue_dense(), poly.enqueue_mc()), max(1, steps // 2))
    return {"workload": f"sierpinski_d{depth}_n{n}", "hop_ms": hop_ms, "mc_ms": mc_ms,
            "ms_per_step": hop_ms + mc_ms, "value": n ** 3 / ((hop_ms + mc_ms) * 1e-3), "unit": "cells/s",
            "dense_ms": dense_ms, "speedup_vs_dense": dense_ms / (hop_ms + mc_ms),
            "counters": {k: c[k] for k in ("n_hop_evals", "n_cand", "n_corner", "n_vert", "n_tri")},
            "evals_per_column": c["n_hop_evals"] / n ** 2, "ops_per_eval": ops_per_eval(recs)}


def cont_section(dev, steps, warmup, recs, n, lo, h, seed):
    """Continuation (gh_cont, the paper's surface-following comparator) on
    the headline workload, seeded with one cell per surface component (found
    from the grid-hopping mesh before timing, as the paper assumes seeds are
    given), followed by marching cubes.  gh_cont waits for each batch of
    levels, so it is timed by the host clock."""
    import numpy as np
    import torch
    from scipy import ndimage

    from paper_2111_05778_amd.polygonize import Bound, Polygonizer, counters_dict
    poly = Polygonizer(Bound.prims(recs, dev), n, lo, h, device=dev, keep_cells=True)
    cells = poly.run().cells.cpu().numpy()
    grid = np.zeros(n ** 3, dtype=bool)
    grid[cells] = True
    lab, k = ndimage.label(grid.reshape(n, n, n))
    flat = lab.reshape(-1)
    seeds = torch.tensor([int(np.flatnonzero(flat == c)[0]) for c in range(1, k + 1)], dtype=torch.int64, device=dev)
    poly.run(seeds=seeds)
    for _ in range(warmup):
        poly.enqueue_cont(seeds)
        poly.enqueue_mc()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(steps):
        levels = poly.enqueue_cont(seeds)
    torch.cuda.synchronize(dev)
    cont_ms = (time.perf_counter() - t0) / steps * 1e3
    mc_ms = event_ms(torch.cuda.current_stream(dev), poly.enqueue_mc, steps)
    c = counters_dict(poly.ctr)
    assert c["flags"] == 0
    return {"workload": f"csg12_seed{seed}_n{n}", "components": int(k), "levels": levels, "cont_ms": cont_ms,
            "mc_ms": mc_ms, "ms_per_step": cont_ms + mc_ms,
            "counters": {kk: c[kk] for kk in ("n_hop_evals", "n_cand", "n_corner", "n_cells", "n_vert", "n_tri")}}


def traced_section(dev, steps, warmup, recs, n, lo, h, seed):
    """The paper's per-column procedure taken literally (gh_hop_traced) on
    the headline workload: its times and counts beside grid hopping's, and
    the audit of sign-change cells it leaves out."""
    import torch
    from paper_2111_05778_amd.polygonize import Bound, Polygonizer, counters_dict
    poly = Polygonizer(Bound.prims(recs, dev), n, lo, h, device=dev, keep_cells=True)
    sign_cells = poly.run().cells.clone()          # grid hopping finds every sign-change cell
    poly.run(traced=True)                          # sizes the buffers for the traced candidates
    for _ in range(warmup):
        poly.enqueue_hop_traced()
        poly.enqueue_mc()
    stream = torch.cuda.current_stream(dev)
    hop_ms = event_ms(stream, poly.enqueue_hop_traced, steps)
    mc_ms = event_ms(stream, poly.enqueue_mc, steps)
    c = counters_dict(poly.ctr)
    assert c["flags"] == 0
    cand = poly.candidates()
    missed = int((~torch.isin(sign_cells, cand)).sum().item())
    return {"workload": f"csg12_seed{seed}_n{n}", "hop_ms": hop_ms, "mc_ms": mc_ms, "ms_per_step": hop_ms + mc_ms,
            "counters": {k: c[k] for k in ("n_hop_evals", "n_cand", "n_corner", "n_cells", "n_vert", "n_tri")},
            "sign_change_cells": int(sign_cells.numel()), "missed_sign_change_cells": missed}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes five times (the known-size kernel "
                         "that scales the HBM counters) and exit")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape autotuner (built-in shapes)")
    ap.add_argument("--sections", default="neural,neural_bf16x3,paper_net,backward,batch,traced,cont,primitives,"
                                          "sierpinski",
                    help="extra workloads to measure after the headline one (comma list, or none)")
    args = ap.parse_args()
    sections = [x for x in args.sections.split(",") if x and x != "none"]
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (each ray column is "
              f"independent: several GPUs would each take a band of columns)", file=sys.stderr)
        sys.exit(2)

    import workloads as W
    n, lo, h = W.grid(args.n)
    recs = W.csg_scene(args.seed)
    # the oracle's legs fork worker processes: before anything touches the GPU
    cpu = None if (args.no_cpu_baseline or args.copy_calibration) else cpu_baseline(recs, n, lo, h)

    import torch

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        x = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize(dev)
        print(json.dumps({"copy_bytes": args.copy_calibration, "launches": 5}), flush=True)
        return

    from paper_2111_05778_amd.polygonize import Bound, Polygonizer

    poly = Polygonizer(Bound.prims(recs, dev), n, lo, h, device=dev, keep_cells=False)
    ref = poly.run()                       # sizes the buffers; reference counters
    c0 = dict(ref.counters)
    tuning = None
    if not args.no_tune:                   # outside the timed region
        from paper_2111_05778_amd import autotune
        tuning, _, _ = autotune.tune(poly, reps=3, store=False)
        poly.tuning = tuning
    stream = torch.cuda.current_stream(dev)

    def timed(enqueue_first, steps, warmup):
        for _ in range(warmup):
            enqueue_first()
            poly.enqueue_mc()
        torch.cuda.synchronize(dev)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for a, b, c in ev:
            a.record(stream)
            enqueue_first()
            b.record(stream)
            poly.enqueue_mc()
            c.record(stream)
        torch.cuda.synchronize(dev)
        wall = time.perf_counter() - t0
        first = [a.elapsed_time(b) * 1e-3 for a, b, _ in ev]
        mc = [b.elapsed_time(c) * 1e-3 for _, b, c in ev]
        return wall, first, mc

    wall, t_hop, t_mc = timed(poly.enqueue_hop, args.steps, args.warmup)
    from paper_2111_05778_amd.polygonize import counters_dict
    c1 = counters_dict(poly.ctr)
    for key in ("n_hop_evals", "n_cand", "n_corner", "n_vert", "n_tri"):
        assert c1[key] == c0[key], (key, c1[key], c0[key])
    assert c1["flags"] == 0

    def graph_wall(dense, steps, warmup):
        # the same step replayed from a captured graph: no host work per kernel
        poly.capture(dense=dense)
        for _ in range(warmup):
            poly.replay()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(steps):
            poly.replay()
        torch.cuda.synchronize(dev)
        return time.perf_counter() - t0

    gwall = graph_wall(False, args.steps, args.warmup)
    c2 = counters_dict(poly.ctr)
    for key in ("n_hop_evals", "n_cand", "n_corner", "n_vert", "n_tri"):
        assert c2[key] == c0[key], (key, c2[key], c0[key])
    assert c2["flags"] == 0

    cells = n ** 3
    ms_per_step = gwall / args.steps * 1e3
    value = cells * args.steps / gwall

    dense = None
    if not args.no_dense:
        dsteps = max(3, args.steps // 4)
        dwall, t_dev, t_dmc = timed(poly.enqueue_dense, dsteps, 1)
        dgwall = graph_wall(True, dsteps, 1)
        dense = {"value": cells * dsteps / dgwall, "ms_per_step": dgwall / dsteps * 1e3,
                 "ms_per_step_eager": dwall / dsteps * 1e3,
                 "eval_ms": 1e3 * sum(t_dev) / len(t_dev), "mc_ms": 1e3 * sum(t_dmc) / len(t_dmc)}

    hop_s = sum(t_hop) / len(t_hop)
    flops = c0["n_hop_evals"] * ops_per_eval(recs)
    achieved = flops / hop_s
    traffic = load_traffic("k_hop")
    roofline = {"bound": "alu", "kernel": "k_hop", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": traffic,
                "peak_issue": PEAK_FP32_ISSUE / 1e12, "frac_issue": achieved / PEAK_FP32_ISSUE,
                "per_launch_flop": flops, "flop_per_eval": ops_per_eval(recs), "hop_ms": hop_s * 1e3,
                "mc_ms": 1e3 * sum(t_mc) / len(t_mc)}

    out = {
        "metric": "grid cells/s polygonized (N\u00b3/t) at N=512 + backward ms; vs dense MC",
        "value": value, "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "ms_per_step_eager": wall / args.steps * 1e3, "launch": "graph",
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"csg12_seed{args.seed}_n{n}", "n": n, "domain": "[-1,1]^3",
                   "primitives": len(recs)},
        "counters": {k: c0[k] for k in ("n_hop_evals", "n_cand", "n_corner", "n_cells", "n_vert", "n_tri")},
        "tuning": tuning,
        "dense": dense,
        "speedup_vs_dense": (dense["ms_per_step"] / ms_per_step) if dense else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    sw = max(1, args.warmup)
    if "neural" in sections:
        out["neural"] = neural_section(dev, max(3, args.steps // 4), sw, dense=not args.no_dense, tune=not args.no_tune)
    if "neural_bf16x3" in sections:
        out["neural_bf16x3"] = neural_section(dev, max(3, args.steps // 4), sw, precision="bf16x3", hop="fp32",
                                              dense=not args.no_dense, tune=not args.no_tune)
    if "paper_net" in sections:
        out["paper_net"] = neural_section(dev, max(3, args.steps // 4), sw, dense=not args.no_dense,
                                          tune=not args.no_tune, paper=True)
    if "backward" in sections:
        out["backward"] = backward_section(dev, max(3, args.steps // 4), sw)
        out["backward_ms"] = out["backward"]["backward_ms"]
    if "batch" in sections:
        out["batch"] = batch_section(dev, max(3, args.steps // 4), sw, tune=not args.no_tune)
    if "cont" in sections:
        out["cont"] = cont_section(dev, max(3, args.steps // 4), sw, recs, n, lo, h, args.seed)
    if "primitives" in sections:
        out["primitives"] = primitives_section(dev, max(3, args.steps // 4), sw)
    if "sierpinski" in sections:
        out["sierpinski"] = sierpinski_section(dev, max(3, args.steps // 4), sw)
    if "traced" in sections:
        out["traced"] = traced_section(dev, max(3, args.steps // 4), sw, recs, n, lo, h, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
