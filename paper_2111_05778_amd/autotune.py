"""Launch-shape autotuner.

The library's launch shapes are process-wide (`gh_set_tuning`): lanes per ray
of the analytic hop and the step budget after which its long rays move to a
pass of one wave and one window of cells per ray, resident blocks per CU of
the marching-cubes look-back scans, list entries per thread of the vertex and
triangle passes, and for the network hop the split policy of tiles with few
rows (waves per group of 32 points), the ray pool of a block (one or two
tiles of rows) and the rows of a draining tile given out as windows of cells
ahead of each ray, and the rays per network work item of a batch.  None of them changes a result, only the time.

`tune()` measures a workload on the device under a coordinate descent over
these shapes: each parameter in turn sweeps its values with the others held
at the best so far; every candidate is timed with HIP events (median of
`reps` runs after one warm-up) and must reproduce the reference counters and
triangles bit for bit, or it is discarded.  The winner is stored in a JSON
cache keyed by device and workload signature (`GH_AUTOTUNE_CACHE`, default
~/.cache/paper_2111_05778_amd/autotune.json) and applied with `apply()`.
"""
import json
import os
import statistics
import tempfile

import torch

from . import native as N

# hop_lanes_per_ray 0 lets the library choose from the bound's type groups.
DEFAULTS = {"hop_lanes_per_ray": 0, "scan_blocks_per_cu": 4, "mlp_split": 3, "batch_rays_per_item": 4096,
            "mc_items_per_thread": 4, "hop_step_budget": 0, "mlp_pool_tiles": 2, "mlp_spec_rows": 32,
            "mlp_lean": 1}
SPACE_PRIMS = {"hop_lanes_per_ray": [0, 1, 2, 3, 4, 8], "hop_step_budget": [0, 32, 64, 128],
               "scan_blocks_per_cu": [1, 2, 4, 8], "mc_items_per_thread": [1, 2, 4, 8]}
SPACE_MLP = {"mlp_split": [1, 2, 3], "mlp_pool_tiles": [1, 2], "mlp_spec_rows": [1, 8, 16, 32],
             "mlp_lean": [1, 2],
             "scan_blocks_per_cu": [1, 2, 4, 8], "mc_items_per_thread": [1, 2, 4, 8]}
SPACE_BATCH = {"batch_rays_per_item": [1024, 2048, 4096, 8192, 16384], "mlp_pool_tiles": [1, 2],
               "mlp_spec_rows": [1, 8, 32]}


def cache_path():
    return os.environ.get("GH_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2111_05778_amd", "autotune.json"))


def load_cache(path=None):
    path = path or cache_path()
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(data, path=None):
    """Atomic replace, so concurrent tuners never leave a torn file."""
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_key(device=None):
    if not torch.cuda.is_available():
        return "cpu"
    p = torch.cuda.get_device_properties(device or torch.cuda.current_device())
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|cu{p.multi_processor_count}"


def signature(spec, n):
    """Workload key: the bound's kind and shape (not its values) and the grid size."""
    if spec.kind == N.GH_SDB_PRIMS:
        types = [0] * N.GH_PRIM_TYPES
        for q in range(spec.n_prim):
            t = spec.prims_h[q * N.GH_PRIM_FLOATS]
            if not (t == int(t) and 0 <= int(t) < N.GH_PRIM_TYPES):
                raise ValueError(f"record {q} has type {t}, not an integer in [0, {N.GH_PRIM_TYPES})")
            types[int(t)] += 1
        return f"prims:{'-'.join(map(str, types))}:n{int(n)}"
    return f"mlp:w{spec.width}:d{spec.depth}:f{spec.n_freq}:p{spec.precision}:n{int(n)}"


def batch_signature(items):
    return "batch:" + ",".join(sorted(signature(b.spec, n) for (b, n) in items))


def full(tuning):
    """Every field resolved (zero or missing means the built-in default)."""
    out = dict(DEFAULTS)
    out.update({k: int(v) for k, v in (tuning or {}).items() if k in DEFAULTS and int(v) != 0})
    return out


def apply(tuning):
    N.gh_set_tuning(**full(tuning))


def lookup(key, device=None, path=None):
    return load_cache(path).get(device_key(device), {}).get(key)


def _median_ms(run, reps, stream):
    run()  # warm-up
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        run()
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def coordinate_descent(space, measure, start=None):
    """Minimises measure(tuning) -> (ms, ok) one parameter at a time."""
    best = full(start)
    best_ms, ok = measure(best)
    if not ok:
        raise RuntimeError("the starting launch shapes do not reproduce the reference")
    trials = [(dict(best), best_ms)]
    for name, values in space.items():
        for v in values:
            if v == best[name]:
                continue
            cand = dict(best)
            cand[name] = v
            ms, ok = measure(cand)
            trials.append((dict(cand), ms if ok else None))
            if ok and ms < best_ms:
                best, best_ms = cand, ms
    return best, best_ms, trials


def tune(poly, reps=5, space=None, store=True, path=None):
    """Tunes the hop + marching-cubes sequence of a Polygonizer (whose buffers
    are already sized, e.g. by one run()).  Returns (tuning, ms, trials)."""
    stream = torch.cuda.current_stream(poly.device)
    if space is None:
        space = SPACE_PRIMS if poly.bound.spec.kind == N.GH_SDB_PRIMS else SPACE_MLP
    saved, saved_poly = N.gh_get_tuning(), poly.tuning
    poly.tuning = None  # the candidates are applied here, not by the Polygonizer

    def run():
        poly.enqueue_hop()
        poly.enqueue_mc()

    apply(None)
    run()
    torch.cuda.synchronize(poly.device)
    ref_ctr = poly.ctr.clone()
    nt = int(ref_ctr[5])
    ref_tris = poly.tris[:nt].clone()

    def measure(t):
        apply(t)
        ms = _median_ms(run, reps, stream)
        ok = torch.equal(poly.ctr, ref_ctr) and torch.equal(poly.tris[:nt], ref_tris)
        return ms, ok

    try:
        best, ms, trials = coordinate_descent(space, measure)
    finally:
        N.gh_set_tuning(**saved)
        poly.tuning = saved_poly
    if store:
        key = signature(poly.bound.spec, poly.n)
        data = load_cache(path)
        data.setdefault(device_key(poly.device), {})[key] = best
        save_cache(data, path)
    return best, ms, trials


def tune_batch(make_batch, items, reps=3, space=SPACE_BATCH, store=True, path=None):
    """Tunes the rays per network work item of a batch.  make_batch() builds a
    BatchPolygonizer (the item list is planned at creation, so each candidate
    needs its own); items: [(Bound, n)] for the cache key."""
    saved = N.gh_get_tuning()
    ref = {}

    def measure(t):
        apply(t)
        batch = make_batch()
        res = batch.run()
        stream = torch.cuda.current_stream(batch.device)
        ms = _median_ms(batch.enqueue, reps, stream)
        got = [(tuple(int(v) for v in p.ctr.tolist()), p.tris[:m.counters["n_tri"]].clone())
               for p, m in zip(batch.polys, res)]
        if not ref:
            ref["v"] = got
        ok = all(a[0] == b[0] and torch.equal(a[1], b[1]) for a, b in zip(got, ref["v"]))
        return ms, ok

    try:
        best, ms, trials = coordinate_descent(space, measure, start=saved)
    finally:
        N.gh_set_tuning(**saved)
    if store:
        data = load_cache(path)
        data.setdefault(device_key(), {})[batch_signature(items)] = best
        save_cache(data, path)
    return best, ms, trials
