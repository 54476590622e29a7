"""Helpers shared by the GPU parity tests: the near-zero exclusion rule for
comparing sign-change cells across precisions, and bands of ray-column rows
cut out of a mesh, so that a full-size GPU mesh can meet the FP64 oracle on
the columns the oracle computes."""
import numpy as np

from oracle import hop as ohop
from oracle import mc as omc

# triangles per marching-cubes case, from the oracle's construction
TRI_COUNT = np.array([len(omc.cell_triangles(c)) for c in range(256)], dtype=np.int64)


def near_zero_mask(f64_at, n, lo, h, cells, thr):
    """For each cell, whether one of its 8 corners has |f64| < thr; f64_at
    takes lattice points (m x 3, FP64) to bound values."""
    cells = np.asarray(cells, dtype=np.int64)
    if len(cells) == 0:
        return np.zeros(0, dtype=bool)
    n1 = n + 1
    pid = ohop.corner_points(n, cells)
    a, b, c = pid // (n1 * n1), (pid // n1) % n1, pid % n1
    P = np.stack([omc.lattice_coords_f64(n, lo, h, v) for v in (a, b, c)], axis=1)
    near = pid[np.abs(f64_at(P)) < thr]
    i, j, k = cells // (n * n), (cells // n) % n, cells % n
    hit = np.zeros(len(cells), dtype=bool)
    for dx, dy, dz in omc.CORNER:
        hit |= np.isin(((i + dx) * n1 + (j + dy)) * n1 + (k + dz), near)
    return hit


def fp32_threshold(P, net, n, lo, h, cells):
    """Exclusion threshold for a network's FP32 signs: four times the largest
    |f32 - f64| over the corners of the given cells, with f32 from the
    library's FP32 evaluator (P is the polygonize module), and at least
    max(1e-6 h, 2^-20)."""
    import torch

    from oracle import sdb as osdb
    n1 = n + 1
    pid = ohop.corner_points(n, cells)
    X = np.stack([omc.lattice_coords_f64(n, lo, h, v) for v in (pid // (n1 * n1), (pid // n1) % n1, pid % n1)],
                 axis=1)
    f32 = P.Bound.mlp(net, "fp32").eval(torch.from_numpy(X.astype(np.float32)).cuda()).cpu().numpy()
    err = float(np.abs(f32 - osdb.neural_f64(net, X)).max()) if len(X) else 0.0
    return max(1e-6 * float(h), 2.0 ** -20, 4 * err)


def assert_cells_match_excluding_near_zero(gpu_cells, gpu_cases, ref_cells, ref_cases, f64_at, n, lo, h, thr,
                                           label=""):
    """Sign-change cells and case bytes equal once cells with a corner
    |f64| < thr are set aside on both sides; returns the set-aside count."""
    ga, gc = np.asarray(gpu_cells), np.asarray(gpu_cases)
    oa, oc = np.asarray(ref_cells), np.asarray(ref_cases)
    union = np.union1d(ga, oa)
    near = union[near_zero_mask(f64_at, n, lo, h, union, thr)]
    kg, ko = ~np.isin(ga, near), ~np.isin(oa, near)
    print(f"{label}: gpu {len(ga)} cells, oracle {len(oa)}, set aside {len(near)} (|f64| < {thr:.2e}), "
          f"differing {len(np.setxor1d(ga, oa))}", flush=True)
    np.testing.assert_array_equal(ga[kg], oa[ko])
    np.testing.assert_array_equal(gc[kg], oc[ko])
    return len(near)


def band_columns(n, i0, i1):
    """Ray columns (i, j) with i0 <= i < i1."""
    return np.arange(i0 * n, i1 * n, dtype=np.int64)


def gpu_band(cells, cases, verts, tris, n, i0, i1):
    """The part of a GPU mesh in the cells with i0 <= i < i1: its cells,
    cases, and a compact (positions, triangles) over the vertices they use.
    Triangles come grouped by cell in cell-id order, so the band's are one
    contiguous range."""
    cells, cases = np.asarray(cells), np.asarray(cases)
    lo_id, hi_id = i0 * n * n, i1 * n * n
    a, b = np.searchsorted(cells, lo_id), np.searchsorted(cells, hi_id)
    counts = TRI_COUNT[cases.astype(np.int64)]
    t0, t1 = int(counts[:a].sum()), int(counts[:b].sum())
    T = np.asarray(tris, dtype=np.int64)[t0:t1]
    used, T = np.unique(T, return_inverse=True)
    return cells[a:b], cases[a:b], np.asarray(verts, dtype=np.float64)[used], T.reshape(-1, 3)


def oracle_band(S, n, lo, h, i0, i1):
    """The FP64 oracle's grid hopping on the band's columns and marching
    cubes on their candidates."""
    cells, evals, col_evals = ohop.hop(S, n, lo, h, columns=band_columns(n, i0, i1))
    return ohop.polygonize_cells(S, n, lo, h, cells, evals, col_evals)
