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
    """Vertices plus seeded barycentric samples on every triangle."""
    rng = np.random.default_rng(seed)
    a, b, c = P[tris[:, 0]], P[tris[:, 1]], P[tris[:, 2]]
    pts = [P]
    for _ in range(per_tri):
        u, v = rng.random(len(tris)), rng.random(len(tris))
        flip = u + v > 1
        u[flip], v[flip] = 1 - u[flip], 1 - v[flip]
        pts.append(a + u[:, None] * (b - a) + v[:, None] * (c - a))
    return np.concatenate(pts)


def hausdorff(PA, TA, PB, TB, per_tri=3):
    """Symmetric Hausdorff distance, estimated from vertex and triangle samples
    of each mesh against the samples of the other."""
    SA, SB = surface_samples(PA, TA, per_tri), surface_samples(PB, TB, per_tri)
    dab = cKDTree(SB).query(SA)[0].max() if len(SA) and len(SB) else np.inf
    dba = cKDTree(SA).query(SB)[0].max() if len(SA) and len(SB) else np.inf
    return max(dab, dba)
