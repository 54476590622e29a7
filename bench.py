"""Benchmark: grid cells polygonized per second (N^3 / t) by grid hopping.

One step = gh_hop + gh_mc over the whole grid (hop over all N^2 ray columns,
distinct corner evaluation, welded vertex and triangle emit) with every
input already resident in HBM.  Workload: min-union of 12 seeded
primitives (sphere, box, torus, capsule; seed 0) on [-1, 1]^3 at N = 512,
float32.  The enumeration path (bound at all (N+1)^3 lattice points,
marching cubes on every cell, same emit) is timed beside it.

Prints one JSON line.  Extra objects:
  roofline      the hop kernel against the FP32 VALU peak of the chip
  cpu_baseline  the oracle (FP64 numpy, one thread) on the same workload
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 FP32 lanes per clock x 2.4 GHz = 39.3e12 FP32 operations/s
# without FMA and without packed dual-FP32 (the published 157.3 TFLOP/s counts
# an FMA as two operations and packed math as two more).
PEAK_FP32_OPS = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12

# FP32 operations per evaluation of each primitive type, counted from the
# formula in include/gh.h (add, sub, mul, min, max, abs, neg, sqrt each 1):
# translate 3 + rotate 15 = 18 shared, then
#   sphere  3 mul + 2 add + sqrt + sub                          = 7
#   box     3 abs + 3 sub + 2 max + 3 max + 3 mul + 2 add + sqrt + min + add = 19
#   torus   2 mul + add + sqrt + sub, 2 mul + add + sqrt + sub  = 10
#   capsule neg + max + min + sub + 3 mul + 2 add + sqrt + sub = 11
#   plane   3 mul + 2 add + sub (no translate/rotate)          = 6 total
#   boxbound 3 abs + 3 sub + 2 max                              = 8
OPS = {0: 18 + 7, 1: 18 + 19, 2: 18 + 10, 3: 18 + 11, 4: 6, 5: 18 + 8}


def ops_per_eval(records):
    types = [int(r[0]) for r in records]
    return sum(OPS[t] for t in types) + (len(types) - 1)   # plus the union minima


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("gh_kernels.hip", "gh_device.h"):
        with open(os.path.join(ROOT, "paper_2111_05778_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel):
    """HBM bytes per launch from the committed PMC summary, if it was taken on
    the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    e = t.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e["bytes_per_launch"]


def cpu_baseline(recs, n, lo, h):
    """The oracle as it stands: FP64 grid hopping + marching cubes, one thread."""
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
    t = min(times)
    return {"value": n ** 3 / t, "unit": "cells/s", "cores": 1, "kind": "oracle",
            "sample": f"the full workload (N={n}, all {n * n} columns), best of 2 runs, {t:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (each ray column is "
              f"independent, the multi-GPU split is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2111_05778_amd.polygonize import Bound, Polygonizer

    dev = torch.device("cuda:0")
    n, lo, h = W.grid(args.n)
    recs = W.csg_scene(args.seed)
    poly = Polygonizer(Bound.prims(recs, dev), n, lo, h, device=dev, keep_cells=False)
    ref = poly.run()                       # sizes the buffers; reference counters
    c0 = dict(ref.counters)
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

    cells = n ** 3
    ms_per_step = wall / args.steps * 1e3
    value = cells * args.steps / wall

    dense = None
    if not args.no_dense:
        dwall, t_dev, t_dmc = timed(poly.enqueue_dense, max(3, args.steps // 4), 1)
        dsteps = max(3, args.steps // 4)
        dense = {"value": cells * dsteps / dwall, "ms_per_step": dwall / dsteps * 1e3,
                 "eval_ms": 1e3 * sum(t_dev) / len(t_dev), "mc_ms": 1e3 * sum(t_dmc) / len(t_dmc)}

    hop_s = sum(t_hop) / len(t_hop)
    flops = c0["n_hop_evals"] * ops_per_eval(recs)
    achieved = flops / hop_s
    traffic = load_traffic("k_hop")
    roofline = {"bound": "alu", "kernel": "k_hop", "achieved": achieved / 1e12, "peak": PEAK_FP32_OPS / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_OPS, "traffic": traffic,
                "per_launch_ops": flops, "ops_per_eval": ops_per_eval(recs), "hop_ms": hop_s * 1e3,
                "mc_ms": 1e3 * sum(t_mc) / len(t_mc)}

    out = {
        "metric": "grid cells/s polygonized (N^3/t) at N=512",
        "value": value, "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"csg12_seed{args.seed}_n{n}", "n": n, "domain": "[-1,1]^3",
                   "primitives": len(recs)},
        "counters": {k: c0[k] for k in ("n_hop_evals", "n_cand", "n_corner", "n_cells", "n_vert", "n_tri")},
        "dense": dense,
        "speedup_vs_dense": (dense["ms_per_step"] / ms_per_step) if dense else None,
        "roofline": roofline,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(recs, n, lo, h),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
