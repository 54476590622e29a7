"""Continuation: the surface-following comparator of the paper (Section 2,
"cont"), test infrastructure like the rest of this package.

From seed cells the search moves to the face neighbours of every cell it
holds whose shared face has a sign change among its four corners (the
surface crosses that face, so the neighbour holds the surface too), until no
new cell appears.  Every cell it reaches is a sign-change cell, and it
reaches all sign-change cells of each surface component that holds a seed.
Lattice values are evaluated once per distinct corner point of the cells
reached.  Level by level (breadth first), which fixes nothing about the
result: the set reached does not depend on the order.

precision "f32" evaluates the bound's FP32 twin at float32 lattice
coordinates (as `mc.enumerate_mesh` does), "f64" the FP64 bound.
"""
import numpy as np

from . import mc

# corner c = dx + 2 dy + 4 dz of a cell; the four corners of each face and
# the neighbour across it
_FACES = [((0, 2, 4, 6), (-1, 0, 0)), ((1, 3, 5, 7), (1, 0, 0)),
          ((0, 1, 4, 5), (0, -1, 0)), ((2, 3, 6, 7), (0, 1, 0)),
          ((0, 1, 2, 3), (0, 0, -1)), ((4, 5, 6, 7), (0, 0, 1))]


def cont(sdb, n, lo, h, seeds, precision="f32"):
    """Cells reached from the seed cell ids, sorted, and the number of
    distinct lattice points evaluated."""
    n1 = n + 1
    visited = np.zeros(n ** 3, dtype=bool)
    known = np.zeros(n1 ** 3, dtype=bool)
    value = np.zeros(n1 ** 3, dtype=np.float64)
    seeds = np.asarray(seeds, dtype=np.int64)
    front = np.unique(seeds[(seeds >= 0) & (seeds < n ** 3)])
    visited[front] = True
    while front.size:
        i, j, k = front // (n * n), (front // n) % n, front % n
        pid = np.stack([((i + dx) * n1 + (j + dy)) * n1 + (k + dz) for (dx, dy, dz) in mc.CORNER], axis=1)
        new = np.unique(pid[~known[pid]])
        if new.size:
            a, b, c = new // (n1 * n1), (new // n1) % n1, new % n1
            if precision == "f64":
                P = np.stack([mc.lattice_coords_f64(n, lo, h, v) for v in (a, b, c)], axis=1)
                value[new] = sdb.f64(P)
            else:
                xs = [mc.lattice_coords_f32(n, lo, h, v) for v in (a, b, c)]
                value[new] = sdb.f32(*xs).astype(np.float64)
            if not np.all(np.isfinite(value[new])):
                raise FloatingPointError("non-finite distance bound value")
            known[new] = True
        neg = value[pid] < 0                          # rows: cells, columns: corners 0..7
        nxt = []
        for corners, (di, dj, dk) in _FACES:
            s = neg[:, corners].sum(axis=1)
            cross = (s > 0) & (s < 4)
            ni, nj, nk = i + di, j + dj, k + dk
            ok = cross & (ni >= 0) & (ni < n) & (nj >= 0) & (nj < n) & (nk >= 0) & (nk < n)
            nxt.append((ni[ok] * n + nj[ok]) * n + nk[ok])
        cand = np.unique(np.concatenate(nxt)) if nxt else np.zeros(0, np.int64)
        front = cand[~visited[cand]]
        visited[front] = True
    return np.nonzero(visited)[0].astype(np.int64), int(known.sum())
