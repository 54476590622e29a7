"""Pins of the oracle's per-cell marching-cubes construction and enumeration.

The construction is checked against facts that do not depend on it: the
crossing edges of a cell are fixed by its corner signs, a single cut corner
is a single triangle facing away from the inside, a plane is reproduced
exactly by linear interpolation, and a closed surface must come out
watertight and consistently oriented on random grids (which are full of
ambiguous faces).
"""
import itertools

import numpy as np
import pytest

from oracle import mc, mesh


def _midpoint(e):
    _, a, b = mc.EDGES[e]
    return (mc.CORNER[a] + mc.CORNER[b]) / 2.0


def test_edge_table_geometry():
    # 12 distinct unit edges of the cube, 4 per axis
    seen = set()
    for axis, a, b in mc.EDGES:
        d = mc.CORNER[b] - mc.CORNER[a]
        assert d.tolist() == [int(i == axis) for i in range(3)]
        seen.add((a, b))
    assert len(seen) == 12
    # each face ring is a 4-cycle of adjacent corners, counter-clockwise seen from outside
    for ring in mc.FACES:
        pts = mc.CORNER[ring].astype(float)
        normal = np.cross(pts[1] - pts[0], pts[2] - pts[1])
        centre = pts.mean(axis=0)
        assert np.dot(normal, centre - 0.5) > 0        # points out of the cube


@pytest.mark.parametrize("case", range(256))
def test_case_uses_exactly_the_crossing_edges(case):
    tris = mc.cell_triangles(case)
    used = sorted({e for t in tris for e in t})
    assert used == mc.crossing_edges(case)
    # every crossing edge lies on exactly one loop, once
    flat = [e for l in mc.cell_loops(case) for e in l]
    assert sorted(flat) == mc.crossing_edges(case)
    assert len(tris) <= 5


def test_table_totals():
    assert mc.cell_triangles(0) == () and mc.cell_triangles(255) == ()
    assert max(len(mc.cell_triangles(c)) for c in range(256)) == 5


@pytest.mark.parametrize("corner", range(8))
def test_single_corner_is_one_outward_triangle(corner):
    for case, inside_corner in ((1 << corner, True), (255 ^ (1 << corner), False)):
        tris = mc.cell_triangles(case)
        assert len(tris) == 1
        a, b, c = (_midpoint(e) for e in tris[0])
        nrm = np.cross(b - a, c - a)
        away = (a + b + c) / 3 - mc.CORNER[corner]
        # facing from inside to outside: away from a lone inside corner,
        # towards a lone outside corner
        assert (np.dot(nrm, away) > 0) == inside_corner


def test_face_of_four_inside_is_a_planar_quad_facing_out():
    case = sum(1 << c for c in range(8) if mc.CORNER[c][2] == 0)   # bottom face inside
    tris = mc.cell_triangles(case)
    assert len(tris) == 2
    for t in tris:
        a, b, c = (_midpoint(e) for e in t)
        assert a[2] == b[2] == c[2] == 0.5
        assert np.cross(b - a, c - a)[2] > 0                          # towards the outside (+z)


def test_ambiguous_face_separates_inside_corners():
    # corners 0 and 3 (diagonal of the z = 0 face) inside: two separate corner cuts
    case = (1 << 0) | (1 << 3)
    tris = mc.cell_triangles(case)
    assert len(mc.cell_loops(case)) == 2 and len(tris) == 2
    for t in tris:
        ends = {c for e in t for c in mc.EDGES[e][1:]}
        assert len(ends & {0, 3}) == 1


def test_plane_reproduced_exactly():
    # linear interpolation along edges puts every vertex exactly on a plane
    n, lo, h = 12, -1.0, 2.0 / 12
    normal = np.array([0.3, -0.5, 0.81])
    normal /= np.linalg.norm(normal)
    ax = lo + np.arange(n + 1) * h
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    F = normal[0] * X + normal[1] * Y + normal[2] * Z - 0.0731
    m = mc.mesh_from_lattice(F, n, lo, h)
    P = m.positions()
    assert len(P) > 50
    np.testing.assert_allclose(P @ normal - 0.0731, 0.0, atol=1e-12)
    # every triangle faces along +normal (from negative to positive side)
    T = m.tri_vertex_index()
    nrm = np.cross(P[T[:, 1]] - P[T[:, 0]], P[T[:, 2]] - P[T[:, 0]])
    assert np.all(nrm @ normal > 0)


@pytest.mark.parametrize("n,seed", [(2, 0), (3, 1), (4, 2), (5, 3), (6, 4), (8, 5)])
def test_random_fields_give_closed_oriented_surfaces(n, seed):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((n + 1,) * 3)
    F[0, :, :] = F[-1, :, :] = F[:, 0, :] = F[:, -1, :] = F[:, :, 0] = F[:, :, -1] = 1.0
    F[F == 0] = 1.0
    m = mc.mesh_from_lattice(F, n, -1.0, 2.0 / n)
    T = m.tri_vertex_index()
    assert len(T) > 0
    assert mesh.is_closed_oriented(T)
    assert mesh.euler_characteristic(T) % 2 == 0
    assert mesh.volume(m.positions(), T) > 0
    # the grids actually exercise ambiguous faces
    amb = 0
    for c in m.cases:
        for ring in mc.FACES:
            s = [(int(c) >> q) & 1 for q in ring]
            amb += s in ([1, 0, 1, 0], [0, 1, 0, 1])
    if n >= 4:
        assert amb > 0


def test_brute_force_single_cells_against_segment_rule():
    # independent re-derivation on each face: crossing edges of the face come in
    # pairs joined by the loops, and a face with two crossings joins exactly those two
    for case in range(256):
        loops = mc.cell_loops(case)
        succ = {}
        for l in loops:
            for a, b in zip(l, l[1:] + l[:1]):
                succ[a] = b
        for ring in mc.FACES:
            fe = [mc._edge_between(ring[p], ring[(p + 1) % 4]) for p in range(4)]
            cross = [e for e in fe if e in succ]
            joined = [(a, succ[a]) for a in cross if succ[a] in fe]
            assert len(joined) == len(cross) // 2
            if len(cross) == 2:
                assert set(joined[0]) == set(cross)


def test_mesh_canonical_form_is_rotation_invariant():
    t = np.array([[5, 2, 9], [9, 5, 2], [2, 9, 5]])
    c = mc.canonical_tris(t)
    assert (c == [2, 9, 5]).all()


def test_edge_ids_and_positions():
    n, lo, h = 4, -1.0, 0.5
    # lattice point (1, 2, 3), axis y, t = 0.25
    eid = 3 * ((1 * 5 + 2) * 5 + 3) + 1
    P = mc.edge_positions(n, lo, h, np.array([eid]), np.array([0.25]))
    np.testing.assert_allclose(P[0], [-0.5, 0.0 + 0.125, 0.5])


def test_all_cases_closed_when_embedded():
    # every case, surrounded by outside corners on a 3^3 grid, closes up
    for case in itertools.islice(range(1, 255), 0, None, 7):
        F = np.ones((4, 4, 4))
        for c in range(8):
            if (case >> c) & 1:
                F[1 + mc.CORNER[c][0], 1 + mc.CORNER[c][1], 1 + mc.CORNER[c][2]] = -1.0
        m = mc.mesh_from_lattice(F, 3, 0.0, 1.0)
        assert mesh.is_closed_oriented(m.tri_vertex_index())
