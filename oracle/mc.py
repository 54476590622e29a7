"""Marching cubes per cell, built from the cell's corner signs (no lookup table),
and enumeration: the same construction applied to every cell of the grid.

The paper polygonizes each reached cell with marching cubes (Section 5) and
says every method yields exactly the same mesh; it leaves the per-cell
construction and the ambiguous faces open.  The construction used here:

  * corner c = dx + 2 dy + 4 dz sits at (dx, dy, dz); it is "inside" when
    f < 0 (negative inside, Section 1; f = 0 counts as outside);
  * edge e joins two corners that differ along one axis: e = 4*axis + r,
    where r enumerates the two other offsets (the lower-numbered axis first);
  * on each of the six faces, walk the four corners counter-clockwise seen
    from outside the cell; every maximal run of inside corners yields one
    segment from the edge where the walk enters the run to the edge where it
    leaves it.  An ambiguous face (inside corners on a diagonal) therefore
    separates the inside corners;
  * each crossing edge starts exactly one segment and ends exactly one, so
    the segments close into loops; each loop is fan-triangulated from its
    smallest edge index.  Triangles then face from inside to outside.

Neighbouring cells walk a shared face in opposite directions over the same
corner signs, so they cut it with the same segments: the mesh is watertight.

Vertex on lattice edge a -> b (a the lower lattice index): t = f_a/(f_a - f_b),
v = P_a + t (P_b - P_a).  Vertices are keyed by the lattice edge id
3*((i*(N+1) + j)*(N+1) + k) + axis of their lower endpoint (i, j, k).
"""
from functools import lru_cache

import numpy as np

# corner c -> (dx, dy, dz)
CORNER = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.int64)


def _edge_table():
    """edge e -> (axis, lower corner, upper corner)."""
    out = []
    for axis in range(3):
        others = [a for a in range(3) if a != axis]
        for r in range(4):
            off = [0, 0, 0]
            off[others[0]] = r & 1
            off[others[1]] = r >> 1
            lo = off[0] + 2 * off[1] + 4 * off[2]
            up = lo + (1 << axis)
            out.append((axis, lo, up))
    return out


EDGES = _edge_table()


def _edge_between(c1, c2):
    for e, (_, a, b) in enumerate(EDGES):
        if {a, b} == {c1, c2}:
            return e
    raise ValueError("corners are not adjacent")


def _faces():
    """Each face as its four corners in counter-clockwise order seen from outside."""
    faces = []
    for axis in range(3):
        u, v = (axis + 1) % 3, (axis + 2) % 3      # e_u x e_v = e_axis
        for side in (0, 1):
            ring = []
            for (du, dv) in ((0, 0), (1, 0), (1, 1), (0, 1)):
                d = [0, 0, 0]
                d[axis], d[u], d[v] = side, du, dv
                ring.append(d[0] + 2 * d[1] + 4 * d[2])
            if side == 0:                           # outward normal is -e_axis
                ring = ring[::-1]
            faces.append(ring)
    return faces


FACES = _faces()


@lru_cache(maxsize=None)
def cell_loops(case):
    """Closed loops of crossing edges for an 8-bit inside mask `case`."""
    inside = [(case >> c) & 1 for c in range(8)]
    nxt = {}
    for ring in FACES:
        s = [inside[c] for c in ring]
        if all(s) or not any(s):
            continue
        for p in range(4):
            # a run of inside corners begins at ring[p] when its predecessor is outside
            if s[p] and not s[p - 1]:
                enter = _edge_between(ring[p - 1], ring[p])
                q = p
                while s[(q + 1) % 4]:
                    q += 1
                leave = _edge_between(ring[q % 4], ring[(q + 1) % 4])
                if enter in nxt:
                    raise AssertionError("edge starts two segments")
                nxt[enter] = leave
    loops, seen = [], set()
    for e0 in sorted(nxt):
        if e0 in seen:
            continue
        loop, e = [], e0
        while e not in seen:
            seen.add(e)
            loop.append(e)
            e = nxt[e]
        if e != e0:
            raise AssertionError("segments do not close into a loop")
        loops.append(loop)
    return tuple(tuple(l) for l in loops)


@lru_cache(maxsize=None)
def cell_triangles(case):
    """Triangles (edge index triples) of a cell: fan of each loop from its smallest edge."""
    tris = []
    for loop in cell_loops(case):
        m = loop.index(min(loop))
        l = loop[m:] + loop[:m]
        for i in range(1, len(l) - 1):
            tris.append((l[0], l[i], l[i + 1]))
    return tuple(tris)


def crossing_edges(case):
    """Edges whose two corners lie on different sides."""
    return [e for e, (_, a, b) in enumerate(EDGES) if ((case >> a) & 1) != ((case >> b) & 1)]


# ------------------------------------------------------------------------ mesh
class Mesh:
    """Canonical mesh: sign-change cells with their case bytes, vertices keyed
    by lattice edge id with their edge parameter t, and triangles as edge-id
    triples rotated to start at their smallest id (orientation kept), sorted."""

    def __init__(self, n, lo, h, cells, cases, edge_ids, ts, tris):
        self.n, self.lo, self.h = int(n), float(lo), float(h)
        order = np.argsort(cells, kind="stable")
        self.cells = np.asarray(cells, dtype=np.int64)[order]
        self.cases = np.asarray(cases, dtype=np.uint8)[order]
        order = np.argsort(edge_ids, kind="stable")
        self.edge_ids = np.asarray(edge_ids, dtype=np.int64)[order]
        self.ts = np.asarray(ts, dtype=np.float64)[order]
        self.tris = canonical_tris(np.asarray(tris, dtype=np.int64).reshape(-1, 3))

    def positions(self):
        """Vertex positions in edge-id order."""
        return edge_positions(self.n, self.lo, self.h, self.edge_ids, self.ts)

    def tri_vertex_index(self):
        """Triangles as indices into positions()."""
        return np.searchsorted(self.edge_ids, self.tris)


def canonical_tris(tris):
    if len(tris) == 0:
        return tris.reshape(0, 3)
    r = np.argmin(tris, axis=1)
    idx = (r[:, None] + np.arange(3)[None, :]) % 3
    t = np.take_along_axis(tris, idx, axis=1)
    order = np.lexsort((t[:, 2], t[:, 1], t[:, 0]))
    return t[order]


def edge_positions(n, lo, h, edge_ids, ts):
    n1 = n + 1
    pid, axis = edge_ids // 3, edge_ids % 3
    k = pid % n1
    j = (pid // n1) % n1
    i = pid // (n1 * n1)
    P = lo + np.stack([i, j, k], axis=1).astype(np.float64) * h
    P[np.arange(len(ts)), axis] += ts * h
    return P


def polygonize(n, lo, h, cells, corner_value):
    """Marching cubes on the given cells.

    cells: int64 ids (i*N + j)*N + k.  corner_value(i, j, k) -> f at lattice
    point P(i, j, k) for integer arrays.  Cells whose corners all lie on one
    side produce nothing and are dropped from the result.
    """
    cells = np.unique(np.asarray(cells, dtype=np.int64))
    i, j, k = cells // (n * n), (cells // n) % n, cells % n
    fc = np.stack([corner_value(i + CORNER[c, 0], j + CORNER[c, 1], k + CORNER[c, 2]) for c in range(8)], axis=1)
    inside = (fc < 0).astype(np.int64)
    case = (inside << np.arange(8)[None, :]).sum(axis=1)
    sc = (case != 0) & (case != 255)
    cells, i, j, k, fc, case = cells[sc], i[sc], j[sc], k[sc], fc[sc], case[sc]
    n1 = n + 1

    def edge_id(e):
        axis, a, _ = EDGES[e]
        pi, pj, pk = i + CORNER[a, 0], j + CORNER[a, 1], k + CORNER[a, 2]
        return 3 * ((pi * n1 + pj) * n1 + pk) + axis

    eids = [edge_id(e) for e in range(12)]
    vert_e, vert_t, tris = [], [], []
    for cs in np.unique(case):
        sel = np.nonzero(case == cs)[0]
        for e in crossing_edges(int(cs)):
            _, a, b = EDGES[e]
            fa, fb = fc[sel, a], fc[sel, b]
            vert_e.append(eids[e][sel])
            vert_t.append(fa / (fa - fb))
        for (e0, e1, e2) in cell_triangles(int(cs)):
            tris.append(np.stack([eids[e0][sel], eids[e1][sel], eids[e2][sel]], axis=1))
    if vert_e:
        ve, vt = np.concatenate(vert_e), np.concatenate(vert_t)
        ve, first = np.unique(ve, return_index=True)
        vt = vt[first]
        tr = np.concatenate(tris)
    else:
        ve, vt, tr = np.zeros(0, np.int64), np.zeros(0), np.zeros((0, 3), np.int64)
    return Mesh(n, lo, h, cells, case, ve, vt, tr)


def lattice_coords_f64(n, lo, h, a):
    return np.float64(lo) + np.asarray(a, dtype=np.float64) * np.float64(h)


def lattice_coords_f32(n, lo, h, a):
    """Float32 lattice coordinate lo + a*h: one rounded product, one rounded sum."""
    return np.float32(lo) + np.asarray(a).astype(np.float32) * np.float32(h)


def enumerate_mesh(sdb, n, lo, h, precision="f64", slab=16):
    """Enumeration (Section 2): f at all (N+1)^3 lattice points, then marching
    cubes on every cell.  This is the definition of the mesh."""
    n1 = n + 1
    ax = np.arange(n1)
    if precision == "f64":
        c = lattice_coords_f64(n, lo, h, ax)
    else:
        c = lattice_coords_f32(n, lo, h, ax)
    F = np.empty((n1, n1, n1), dtype=np.float64)
    X, Y = np.meshgrid(c, c, indexing="ij")
    for k0 in range(0, n1, slab):
        ks = c[k0:k0 + slab]
        x = np.broadcast_to(X[:, :, None], (n1, n1, len(ks)))
        y = np.broadcast_to(Y[:, :, None], (n1, n1, len(ks)))
        z = np.broadcast_to(ks[None, None, :], (n1, n1, len(ks)))
        if precision == "f64":
            P = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
            F[:, :, k0:k0 + slab] = sdb.f64(P).reshape(n1, n1, len(ks))
        else:
            F[:, :, k0:k0 + slab] = sdb.f32(x.ravel(), y.ravel(), z.ravel()).astype(np.float64).reshape(n1, n1, len(ks))
    return mesh_from_lattice(F, n, lo, h), F


def mesh_from_lattice(F, n, lo, h):
    """Marching cubes over every cell of a lattice of values F[(N+1)^3]."""
    neg = F < 0
    case = np.zeros((n, n, n), dtype=np.int64)
    for c in range(8):
        dx, dy, dz = CORNER[c]
        case |= neg[dx:dx + n, dy:dy + n, dz:dz + n].astype(np.int64) << c
    sc = np.nonzero((case != 0) & (case != 255))
    cells = (sc[0] * n + sc[1]) * n + sc[2]
    return polygonize(n, lo, h, cells, lambda i, j, k: F[i, j, k])
