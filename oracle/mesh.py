"""Mesh checks on triangle meshes given as positions (V x 3) and index triples."""
import numpy as np
from scipy.spatial import cKDTree


def undirected_edges(tris):
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    return np.sort(e, axis=1)


def is_closed_oriented(tris):
    """Every edge is used by exactly two triangles, once in each direction."""
    if len(tris) == 0:
        return True
    d = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    fwd = {tuple(x) for x in d.tolist()}
    if len(fwd) != len(d):
        return False                      # some directed edge repeats
    return all((b, a) in fwd for (a, b) in fwd)


def euler_characteristic(tris):
    """V - E + F over the vertices the triangles reference."""
    v = len(np.unique(tris))
    e = len(np.unique(undirected_edges(tris), axis=0))
    return v - e + len(tris)


def area(P, tris):
    a, b, c = P[tris[:, 0]], P[tris[:, 1]], P[tris[:, 2]]
    return 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1).sum()


def volume(P, tris):
    """Enclosed volume by the divergence theorem (positive for outward faces)."""
    a, b, c = P[tris[:, 0]], P[tris[:, 1]], P[tris[:, 2]]
    return np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0


def surface_samples(P, tris, per_tri=3, seed=0):
    """Points on the mesh: its vertices, the midpoint of every triangle edge,
    every triangle's centroid, and per_tri seeded uniform points per triangle."""
    rng = np.random.default_rng(seed)
    a, b, c = P[tris[:, 0]], P[tris[:, 1]], P[tris[:, 2]]
    pts = [P, 0.5 * (a + b), 0.5 * (b + c), 0.5 * (c + a), (a + b + c) / 3.0]
    for _ in range(per_tri):
        u, v = rng.random(len(tris)), rng.random(len(tris))
        flip = u + v > 1
        u[flip], v[flip] = 1 - u[flip], 1 - v[flip]
        pts.append(a + u[:, None] * (b - a) + v[:, None] * (c - a))
    return np.concatenate(pts)


def _segment_distance(P, A, B):
    """Row-wise distance from P[i] to the segment A[i] B[i] (a point if A = B)."""
    d = B - A
    dd = np.einsum("ij,ij->i", d, d)
    t = np.einsum("ij,ij->i", P - A, d) / np.where(dd > 0, dd, 1.0)
    t = np.clip(np.where(dd > 0, t, 0.0), 0.0, 1.0)
    return np.linalg.norm(P - (A + t[:, None] * d), axis=1)


def point_triangle_distance(P, A, B, C):
    """Row-wise distance from P[i] to the triangle A[i] B[i] C[i]: the height
    above its plane where the foot of the perpendicular falls inside the
    triangle, else the distance to the nearest of its three edges (the only
    candidates then).  A degenerate triangle (zero area) is its edges."""
    u, v, w = B - A, C - A, P - A
    n = np.cross(u, v)
    nn = np.einsum("ij,ij->i", n, n)
    uu, uv, vv = (np.einsum("ij,ij->i", x, y) for x, y in ((u, u), (u, v), (v, v)))
    wu, wv = np.einsum("ij,ij->i", w, u), np.einsum("ij,ij->i", w, v)
    den = uu * vv - uv * uv
    flat = (nn <= 1e-30 * np.maximum(uu * vv, 1e-300)) | (den <= 0)
    safe = np.where(flat, 1.0, den)
    beta = (vv * wu - uv * wv) / safe
    gamma = (uu * wv - uv * wu) / safe
    inside = ~flat & (beta >= 0) & (gamma >= 0) & (beta + gamma <= 1)
    height = np.abs(np.einsum("ij,ij->i", w, n)) / np.sqrt(np.where(flat, 1.0, nn))
    edges = np.minimum(np.minimum(_segment_distance(P, A, B), _segment_distance(P, B, C)),
                       _segment_distance(P, C, A))
    return np.where(inside, height, edges)


def distance_to_mesh(S, P, tris, chunk=200_000):
    """Exact distance from each point of S to the surface of the mesh (P, tris).

    Candidates come from a KD-tree over triangle centroids: a triangle whose
    centroid lies at distance c from a point is at least c - r away from it,
    r the largest centroid-to-vertex distance of any triangle.  With the k
    nearest centroids examined, a point whose best distance is at most the
    k-th centroid distance minus r is exact; the others are redone with more
    candidates, the last round with every triangle within best + r."""
    S = np.asarray(S, dtype=np.float64)
    if len(tris) == 0:
        return np.full(len(S), np.inf)
    A, B, C = P[tris[:, 0]], P[tris[:, 1]], P[tris[:, 2]]
    cen = (A + B + C) / 3.0
    r = np.sqrt(max((np.einsum("ij,ij->i", X - cen, X - cen)).max() for X in (A, B, C)))
    tree = cKDTree(cen)
    out = np.empty(len(S))
    for c0 in range(0, len(S), chunk):
        Q = S[c0:c0 + chunk]
        best = np.full(len(Q), np.inf)
        todo = np.arange(len(Q))
        for k in (8, 32, 128):
            k = min(k, len(tris))
            dist, idx = tree.query(Q[todo], k=k)
            dist, idx = dist.reshape(len(todo), k), idx.reshape(len(todo), k)
            rows = np.repeat(todo, k)
            d = point_triangle_distance(Q[rows], A[idx.ravel()], B[idx.ravel()], C[idx.ravel()])
            best[todo] = np.minimum(best[todo], d.reshape(len(todo), k).min(axis=1))
            exact = (k == len(tris)) | (best[todo] <= dist[:, -1] - r)
            todo = todo[~exact]
            if len(todo) == 0:
                break
        for q in todo:                       # the rest: every triangle that could be nearer
            cand = np.asarray(tree.query_ball_point(Q[q], best[q] + r), dtype=np.int64)
            if len(cand):
                d = point_triangle_distance(np.repeat(Q[q][None], len(cand), 0), A[cand], B[cand], C[cand])
                best[q] = min(best[q], d.min())
        out[c0:c0 + chunk] = best
    return out


def hausdorff_one_sided(PA, TA, PB, TB, per_tri=3):
    """Largest distance from mesh A to the surface of mesh B, over A's
    vertices, edge midpoints, centroids and per_tri seeded points per
    triangle (surface_samples), each measured exactly to B's triangles."""
    SA = surface_samples(PA, TA, per_tri)
    if len(SA) == 0:
        return 0.0
    return float(distance_to_mesh(SA, PB, TB).max())


def hausdorff(PA, TA, PB, TB, per_tri=3):
    """Symmetric Hausdorff distance: the larger of the two one-sided ones."""
    return max(hausdorff_one_sided(PA, TA, PB, TB, per_tri), hausdorff_one_sided(PB, TB, PA, TA, per_tri))
