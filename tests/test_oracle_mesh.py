"""Pins of the oracle's mesh distance (oracle/mesh.py), which checks the
bf16 meshes against the FP64 ones: exact point-to-triangle distances, and
Hausdorff distances with closed-form values (a translated cube, concentric
inscribed polyhedra, a hole, coplanar meshes of different resolution).  Two
planted mistakes, a one-sided measure and a vertex-only one, each fail one
of the pins."""
import numpy as np
from scipy.spatial import cKDTree

from oracle import mesh as M


def grid_patch(m, size=1.0, origin=(0.0, 0.0)):
    """Unit-square patch in z = 0 split into m x m squares, two triangles each."""
    x = origin[0] + np.linspace(0, size, m + 1)
    y = origin[1] + np.linspace(0, size, m + 1)
    X, Y = np.meshgrid(x, y, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    vid = lambda i, j: i * (m + 1) + j  # noqa: E731
    T = []
    for i in range(m):
        for j in range(m):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            T += [(a, b, c), (a, c, d)]
    return P, np.array(T, dtype=np.int64)


def cube_surface(m):
    """Surface of [-1, 1]^3, each face an m x m grid of squares."""
    Ps, Ts, off = [], [], 0
    P0, T0 = grid_patch(m, 2.0, (-1.0, -1.0))
    for axis in range(3):
        for side in (-1.0, 1.0):
            P = np.zeros_like(P0)
            others = [a for a in range(3) if a != axis]
            P[:, others[0]], P[:, others[1]] = P0[:, 0], P0[:, 1]
            P[:, axis] = side
            Ps.append(P)
            Ts.append(T0 + off)
            off += len(P)
    return np.concatenate(Ps), np.concatenate(Ts)


def icosphere(levels, radius):
    t = (1 + 5 ** 0.5) / 2
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    V = [np.array(v, float) / np.linalg.norm(v) for v in V]
    for _ in range(levels):
        mid, F2 = {}, []

        def m_(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                p = V[a] + V[b]
                V.append(p / np.linalg.norm(p))
                mid[key] = len(V) - 1
            return mid[key]
        for a, b, c in F:
            ab, bc, ca = m_(a, b), m_(b, c), m_(c, a)
            F2 += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = F2
    return radius * np.array(V), np.array(F, dtype=np.int64)


def test_point_triangle_distance_regions_and_brute_force():
    A, B, C = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.0, 1, 0])
    cases = {(0.2, 0.2, 0.7): 0.7,                 # above the interior: the height
             (0.5, -0.3, 0.4): 0.5,                # beside edge AB: distance to the edge
             (-0.3, -0.4, 0.0): 0.5,               # beyond vertex A
             (1.0, 1.0, 0.0): 0.5 ** 0.5}          # beyond edge BC
    for p, want in cases.items():
        got = M.point_triangle_distance(np.array([p]), A[None], B[None], C[None])[0]
        assert abs(got - want) < 1e-12, (p, got, want)
    rng = np.random.default_rng(7)
    P, T3 = rng.normal(size=(64, 3)), rng.normal(size=(64, 3, 3))
    exact = M.point_triangle_distance(P, T3[:, 0], T3[:, 1], T3[:, 2])
    g = np.linspace(0, 1, 301)
    U, V = np.meshgrid(g, g, indexing="ij")
    keep = U + V <= 1
    U, V = U[keep], V[keep]
    for q in range(len(P)):
        a, b, c = T3[q]
        S = a + U[:, None] * (b - a) + V[:, None] * (c - a)
        brute = np.linalg.norm(S - P[q], axis=1).min()
        spacing = max(np.linalg.norm(b - a), np.linalg.norm(c - a)) / 300
        assert exact[q] <= brute + 1e-12 and brute - exact[q] <= spacing, (q, exact[q], brute)
    # a triangle of three equal points is a point
    d = M.point_triangle_distance(np.array([[1.0, 2, 2]]), *(np.zeros((1, 3)),) * 3)
    assert abs(d[0] - 3.0) < 1e-12


def test_translated_cube_is_delta_away():
    P, T = cube_surface(6)
    for delta in (0.05, 0.2):
        Q = P + np.array([delta, 0.0, 0.0])
        assert abs(M.hausdorff(P, T, Q, T) - delta) < 1e-12
        assert abs(M.hausdorff_one_sided(P, T, Q, T) - delta) < 1e-12
        assert abs(M.hausdorff_one_sided(Q, T, P, T) - delta) < 1e-12
    assert M.hausdorff(P, T, P, T) == 0.0


def test_concentric_inscribed_polyhedra():
    """An inscribed icosphere of radius r and its copy scaled to r + delta:
    the outer one's vertices are exactly delta from the inner surface (which
    lies below each vertex's tangent plane), every other point is nearer."""
    r, delta = 0.5, 0.03
    P, T = icosphere(2, r)
    Q = P * (r + delta) / r
    assert abs(M.hausdorff_one_sided(Q, T, P, T) - delta) < 1e-12
    inner = M.hausdorff_one_sided(P, T, Q, T)
    assert 0.9 * delta < inner < delta
    assert abs(M.hausdorff(P, T, Q, T) - delta) < 1e-12


def test_hole_is_seen_from_the_full_side_only():
    """A 20 x 20 patch of squares of side 0.05 without the 6 x 6 block around
    its centre: the centre is 0.15 from the rest; the holed patch lies on the
    full one (distance 0)."""
    P, T = grid_patch(20)
    cen = (P[T[:, 0]] + P[T[:, 1]] + P[T[:, 2]]) / 3
    hole = (np.abs(cen[:, 0] - 0.5) < 0.15) & (np.abs(cen[:, 1] - 0.5) < 0.15)
    TH = T[~hole]
    assert abs(M.hausdorff_one_sided(P, T, P, TH) - 0.15) < 1e-12
    assert M.hausdorff_one_sided(P, TH, P, T) == 0.0
    assert abs(M.hausdorff(P, TH, P, T) - 0.15) < 1e-12
    # planted mistake: measuring from the first mesh only misses the hole
    assert M.hausdorff_one_sided(P, TH, P, T) != 0.15


def test_coplanar_meshes_of_different_resolution_coincide():
    """Two triangulations of one square are 0 apart as surfaces; a checker that
    measured to the other mesh's vertices only would report about half a
    coarse square's diagonal."""
    PF, TF = grid_patch(20)
    PC, TC = grid_patch(2)
    assert M.hausdorff(PF, TF, PC, TC) < 1e-12
    # planted mistake: nearest vertex instead of nearest surface point
    vertex_only = cKDTree(PC).query(M.surface_samples(PF, TF))[0].max()
    assert vertex_only > 0.3


def test_distance_to_mesh_exact_when_candidates_run_out():
    """Long thin triangles make the centroid radius large, so the certificate
    fails for the first rounds and the ball search has to finish the job:
    compare with brute force over every triangle."""
    rng = np.random.default_rng(3)
    P = rng.normal(size=(300, 3))
    T = rng.integers(0, len(P), size=(400, 3))
    S = rng.normal(size=(200, 3)) * 1.5
    got = M.distance_to_mesh(S, P, T)
    A, B, C = P[T[:, 0]], P[T[:, 1]], P[T[:, 2]]
    brute = np.array([M.point_triangle_distance(np.repeat(s[None], len(T), 0), A, B, C).min() for s in S])
    np.testing.assert_allclose(got, brute, rtol=0, atol=1e-12)
