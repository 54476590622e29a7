"""Pins of the oracle's grid hopper against the paper's analysis and against
enumeration.

* Plane perpendicular to the rays (Section 4.1, case 1): one approach step,
  then the distance doubles each step; the per-column count has a closed form.
* Plane parallel to the rays (case 2): a column at distance s*h takes
  ceil(N/s) steps; the total is compared with the paper's N^2 (1 + 2 H_N).
* O(N^2 log N) growth (Sections 3-4) versus N^3 for enumeration.
* Grid hopping and enumeration give identical meshes (Section 5).
* A scaled-up function (not a distance bound) makes the hopper miss cells
  (Section 5.2), and the max-of-planes box bound (eq. boxdist) gives the same
  mesh as the exact box distance with more evaluations (Section 4.2).
* Sphere: watertight, Euler characteristic 2, area and volume converge to
  pi and pi/6 at second order.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import hop, mc, mesh, sdb


def _mesh_equal(a, b):
    return (np.array_equal(a.cells, b.cells) and np.array_equal(a.cases, b.cases)
            and np.array_equal(a.tris, b.tris) and np.array_equal(a.edge_ids, b.edge_ids))


@pytest.mark.parametrize("n", [16, 64, 256, 1024])
def test_plane_perpendicular_closed_form(n):
    C = 0.1234
    _, lo, h = W.grid(n)
    lo, h = float(lo), float(h)
    S = sdb.SDB.prims(W.plane_scene((0, 0, 1), C))
    cols = np.arange(0, n * n, max(1, n * n // 64))
    cells, total, per_col = hop.hop(S, n, lo, h, columns=cols)
    # approach: the exact distance lands in the cell holding C in one step
    z0 = lo + 0.5 * h
    k1 = math.floor((C - z0) / h)
    frac = (C - z0) / h - k1
    assert 0 < frac < 1
    # then cells k1 and k1+1 are within h of the plane; afterwards the distance
    # from the plane is (m - frac) h at cell k1 + m, so the steps are 1, 2, 4, ...
    escape = 0
    k = k1 + 2
    while k < n:
        escape += 1
        k += math.floor(k - k1 - frac)
    expected = 1 + 2 + escape
    assert (per_col == expected).all()
    assert expected == round(math.log2(n)) + 2        # doubling: log2 N escape steps
    assert len(cells) == 2 * len(cols)


def test_candidates_within_half_a_diagonal():
    """The candidate test: a cell is marked only when its centroid value is at
    most half the cell's diagonal plus h/32, (sqrt 3 / 2 + 1/32) h.  A plane
    at z = C placed so that the two cells within h of it sit at 0.07 h and
    0.93 h from their centroids: the far one is stepped over, each column
    marks exactly the cell holding the plane, the evaluation count keeps its
    closed form, and the mesh equals enumeration's."""
    n = 64
    _, lo, h = W.grid(n)
    lo, h = float(lo), float(h)
    k1 = 35
    C = lo + (k1 + 0.5 + 0.93) * h
    S = sdb.SDB.prims(W.plane_scene((0, 0, 1), C))
    cells, total, per_col = hop.hop(S, n, lo, h)
    assert (per_col == round(math.log2(n)) + 2).all()
    np.testing.assert_array_equal(cells % n, np.full(n * n, k1 + 1))
    dense, _ = mc.enumerate_mesh(S, n, lo, h)
    assert _mesh_equal(hop.gridhop(S, n, lo, h).mesh, dense)
    # parallel to the rays: columns between the threshold and h from the
    # plane take one evaluation per cell and mark nothing
    T = (np.sqrt(3) / 2 + 1 / 32) * h
    assert np.isclose(hop.candidate_threshold_f64(n, lo, h), T)
    S = sdb.SDB.prims(W.plane_scene((1, 0, 0), C))
    cells, total, per_col = hop.hop(S, n, lo, h)
    xs = lo + (np.arange(n) + 0.5) * h
    dist = np.abs(xs - C)
    assert ((dist > T) & (dist < h)).sum() == 1
    marked = np.unique(cells // (n * n))
    np.testing.assert_array_equal(marked, np.nonzero(dist <= T)[0])
    assert total == n * int(np.where(dist < h, n, np.ceil(n / np.maximum(np.floor(dist / h), 1))).sum())


def test_float32_threshold_margin_keeps_corner_zeros(monkeypatch):
    """The Sierpinski tetrahedron of depth 5 at N = 96 has zeros on lattice
    points, so some sign-change cells hold their zero at a corner, exactly
    half a diagonal from the centroid.  In float32 the centroid value comes
    out a little above (sqrt 3 / 2) h; the h/32 of the threshold keeps those
    cells (the twin's candidates hold every float32 sign-change cell), and a
    threshold of (sqrt 3 / 2) h alone (the planted mistake) loses them."""
    S = sdb.SDB.prims(W.sierpinski_scene(5))
    n, lo, h = W.grid(96)
    dense, _ = mc.enumerate_mesh(S, n, lo, h, precision="f32")
    cells, _, _ = hop.hop(S, n, lo, h, precision="f32")
    assert np.all(np.isin(dense.cells, cells))
    monkeypatch.setattr(hop, "candidate_threshold_f32",
                        lambda nn, ll, hh: np.float32(np.float64(np.float32(hh)) * (np.sqrt(3.0) / 2.0)))
    cells, _, _ = hop.hop(S, n, lo, h, precision="f32")
    assert not np.all(np.isin(dense.cells, cells))


def test_candidate_threshold_on_small_cells():
    # h below 2^-12 of the coordinate scale: every cell with a zero step is
    # a candidate (threshold h); the twin's float32 threshold rounds once
    assert hop.candidate_threshold_f64(64, 1000.0, 1e-3) == 1e-3
    assert hop.candidate_threshold_f64(64, -1.0, 2 / 64) == (np.sqrt(3.0) / 2.0 + 1.0 / 32.0) * (2 / 64)
    t32 = hop.candidate_threshold_f32(512, -1.0, 2 / 512)
    assert t32 == np.float32((np.sqrt(3.0) / 2.0 + 1.0 / 32.0) * np.float64(np.float32(2 / 512)))


@pytest.mark.parametrize("scene", ["sphere", "csg"])
def test_half_diagonal_is_needed(scene, monkeypatch):
    """Planted mistake: a threshold of h / 2 instead of half the diagonal
    leaves sign-change cells whose zero lies towards a corner unmarked, and
    the mesh loses triangles."""
    recs = W.sphere_scene(0.5) if scene == "sphere" else W.csg_scene(1)
    S = sdb.SDB.prims(recs)
    n, lo, h = W.grid(48)
    dense, _ = mc.enumerate_mesh(S, n, lo, h)
    assert _mesh_equal(hop.gridhop(S, n, lo, h).mesh, dense)
    monkeypatch.setattr(hop, "candidate_threshold_f64", lambda nn, ll, hh: 0.5 * np.float64(hh))
    cells, _, _ = hop.hop(S, n, lo, h)
    assert not np.all(np.isin(dense.cells, cells))


@pytest.mark.parametrize("n", [16, 64, 256])
def test_plane_parallel_count_and_harmonic_bound(n):
    C = 0.1234
    _, lo, h = W.grid(n)
    lo, h = float(lo), float(h)
    S = sdb.SDB.prims(W.plane_scene((1, 0, 0), C))
    cells, total, per_col = hop.hop(S, n, lo, h)
    xs = lo + (np.arange(n) + 0.5) * h
    s = np.floor(np.abs(xs - C) / h).astype(int)
    expected_per_x = np.where(s == 0, n, np.ceil(n / np.maximum(s, 1)))
    assert total == n * int(expected_per_x.sum())
    H = sum(1.0 / i for i in range(1, n + 1))
    ratio = total / (n * n * (1 + 2 * H))
    assert 0.9 < ratio < 1.1                          # the paper's estimate is approximate
    # the candidates are exactly the columns whose centre line is within h of x = C
    assert len(cells) == n * n * int((s == 0).sum())


def test_evaluation_count_grows_like_n2_log_n():
    S = sdb.SDB.prims(W.sphere_scene())
    ns = [16, 32, 64, 128, 256]
    per_col = []
    for n in ns:
        _, total, _ = hop.hop(S, *W.grid(n))
        per_col.append(total / n ** 2)
    x = np.log2(ns)
    slope, icpt = np.polyfit(x, per_col, 1)
    pred = slope * x + icpt
    r2 = 1 - ((per_col - pred) ** 2).sum() / ((per_col - np.mean(per_col)) ** 2).sum()
    assert r2 > 0.99
    assert 0.8 < slope < 1.3                          # about one more step per doubling
    # enumeration evaluates (N+1)^3 points, about N per column: the advantage
    # of hopping grows with every doubling of N
    adv = [(n + 1) ** 3 / n ** 2 / c for n, c in zip(ns, per_col)]
    assert np.all(np.diff(adv) > 0) and adv[-1] > 20


def test_general_plane_logarithmic():
    nrm = np.array([0.3, -0.4, -0.866])
    S = sdb.SDB.prims(W.plane_scene(nrm, 0.05))
    vals = [hop.hop(S, *W.grid(n))[1] / n ** 2 for n in (16, 32, 64, 128)]
    d = np.diff(vals)
    assert np.all(d > 0) and np.all(d < 3.0)          # bounded increment per doubling


@pytest.mark.parametrize("scene,n", [("sphere", 16), ("sphere", 64), ("csg0", 32), ("csg1", 64),
                                     ("csg2", 48), ("box", 40)])
def test_hop_equals_enumeration(scene, n):
    recs = {"sphere": W.sphere_scene(), "csg0": W.csg_scene(0), "csg1": W.csg_scene(1),
            "csg2": W.csg_scene(2), "box": W.box_scene((0.31, 0.2, 0.45), (0.05, -0.1, 0.02))}[scene]
    S = sdb.SDB.prims(recs)
    g = W.grid(n)
    dense, _ = mc.enumerate_mesh(S, *g)
    hr = hop.gridhop(S, *g)
    assert len(dense.cells) > 0
    assert _mesh_equal(dense, hr.mesh)
    assert np.isin(dense.cells, hr.candidates).all()
    np.testing.assert_array_equal(dense.ts, hr.mesh.ts)


def test_hop_equals_enumeration_neural():
    S = sdb.SDB.neural(W.neural_scene(0, 64))
    g = W.grid(32)
    dense, _ = mc.enumerate_mesh(S, *g)
    hr = hop.gridhop(S, *g)
    assert _mesh_equal(dense, hr.mesh)
    assert len(dense.cells) > 500


def test_vectorised_hopper_matches_plain_loop():
    recs = W.csg_scene(0)
    S = sdb.SDB.prims(recs)
    n, lo, h = W.grid(32)
    lo, h = float(lo), float(h)
    rng = np.random.default_rng(7)
    cols = rng.choice(n * n, 40, replace=False)
    cells, _, per_col = hop.hop(S, n, lo, h, columns=cols)
    for q, c in enumerate(cols):
        i, j = divmod(int(c), n)
        x, y = lo + (i + 0.5) * h, lo + (j + 0.5) * h

        def f(k):
            return float(sdb.union_f64(recs, np.array([[x, y, lo + (k + 0.5) * h]]))[0])

        ks, ev = hop.hop_column(f, n, h, lo)
        assert ev == per_col[q]
        mine = cells[(cells // n) == c] % n
        assert list(mine) == ks


def test_scaled_function_misses_cells():
    # 2 f overestimates the distance: hops jump over surface cells
    base = sdb.SDB.prims(W.sphere_scene())
    g = W.grid(64)
    dense, _ = mc.enumerate_mesh(base, *g)
    cells, _, _ = hop.hop(base.scaled(2.0), *g)
    missed = np.setdiff1d(dense.cells, cells)
    assert len(missed) > 1000
    # 1/2 f is still a bound: nothing missed, more evaluations
    cells_half, ev_half, _ = hop.hop(base.scaled(0.5), *g)
    _, ev_full, _ = hop.hop(base, *g)
    assert np.isin(dense.cells, cells_half).all() and ev_half > ev_full


def test_box_bound_same_mesh_more_evaluations():
    half, ctr = (0.3, 0.45, 0.2), (0.02, -0.05, 0.11)
    g = W.grid(64)
    exact = hop.gridhop(sdb.SDB.prims(W.box_scene(half, ctr)), *g)
    bound = hop.gridhop(sdb.SDB.prims(W.box_scene(half, ctr, bound=True)), *g)
    assert np.array_equal(exact.mesh.cells, bound.mesh.cells)
    assert np.array_equal(exact.mesh.tris, bound.mesh.tris)
    assert bound.hop_evals > exact.hop_evals


def test_sphere_closed_forms_converge():
    S = sdb.SDB.prims(W.sphere_scene(0.5))
    ea, ev = [], []
    for n in (16, 32, 64, 128):
        m = hop.gridhop(S, *W.grid(n)).mesh
        P, T = m.positions(), m.tri_vertex_index()
        assert mesh.is_closed_oriented(T)
        assert mesh.euler_characteristic(T) == 2
        ea.append(abs(mesh.area(P, T) - math.pi))
        ev.append(abs(mesh.volume(P, T) - math.pi / 6))
        # vertices lie on the sphere up to the interpolation error O(h^2)
        r = np.linalg.norm(P, axis=1)
        assert np.abs(r - 0.5).max() < 0.5 * (2.0 / n) ** 2
    for e in (ea, ev):
        ratios = np.array(e[:-1]) / np.array(e[1:])
        assert np.all((ratios > 3.0) & (ratios < 5.0))   # second order in h


def test_fp32_twin_agrees_with_fp64():
    recs = W.csg_scene(0)
    S = sdb.SDB.prims(recs)
    n, lo, h = W.grid(64)
    rng = np.random.default_rng(0)
    P = rng.uniform(-1, 1, size=(20000, 3)).astype(np.float32)
    f32 = S.f32(P[:, 0], P[:, 1], P[:, 2]).astype(np.float64)
    f64 = S.f64(P.astype(np.float64))
    assert np.abs(f32 - f64).max() < 2e-6
    a = hop.gridhop(S, n, lo, h, precision="f32")
    b = hop.gridhop(S, n, lo, h, precision="f64")
    assert _mesh_equal(a.mesh, b.mesh)
    # t = f_a/(f_a - f_b) amplifies the float32 rounding of f by 1/|f_a - f_b|:
    # nearly all vertices agree to 1e-5 of an edge, none by more than 1e-3
    dt = np.abs(a.mesh.ts - b.mesh.ts)
    assert dt.max() < 1e-3 and (dt > 1e-5).mean() < 1e-3
    # twin centroids are exact for power-of-two grids
    np.testing.assert_array_equal(hop.centroid_f32(lo, h, np.arange(n)).astype(np.float64),
                                  hop.centroid_f64(lo, h, np.arange(n)))


def _near_zero_cells(S, n, lo, h, cells, floor):
    """Cells of the list with a corner whose FP64 value has |f| < floor."""
    n1 = n + 1
    pid = hop.corner_points(n, cells)
    a, b, c = pid // (n1 * n1), (pid // n1) % n1, pid % n1
    P = np.stack([mc.lattice_coords_f64(n, lo, h, v) for v in (a, b, c)], axis=1)
    near = pid[np.abs(S.f64(P)) < floor]
    i, j, k = cells // (n * n), (cells // n) % n, cells % n
    hit = np.zeros(len(cells), dtype=bool)
    for dx, dy, dz in mc.CORNER:
        hit |= np.isin(((i + dx) * n1 + (j + dy)) * n1 + (k + dz), near)
    return cells[hit]


@pytest.mark.slow
@pytest.mark.parametrize("n", [256, 512])
def test_fp32_twin_matches_fp64_at_full_size(n):
    """CSG-12 (seed 0) at the benchmark sizes: the float32 twin, which the GPU
    path equals bit for bit, against the FP64 oracle (Section 3: grid hopping
    polygonizes every cell the surface crosses; Section 5: the same mesh as
    enumeration).  Once cells with a corner |f64| < max(1e-6 h, 2^-20) are set
    aside, the sign-change cells and their case bytes are identical.  The
    set-aside count is printed; a corner of a cell the surface crosses lands
    within the floor of zero with probability about 2 floor/h (|grad f| <= 1),
    so about 16 floor/h of the cells are set aside (0.4 % at N = 512), and
    the test allows twice that."""
    recs = W.csg_scene(0)
    S = sdb.SDB.prims(recs)
    _, lo, h = W.grid(n)
    a = hop.gridhop(S, n, lo, h, precision="f32").mesh
    b = hop.gridhop(S, n, lo, h, precision="f64").mesh
    floor = max(1e-6 * h, 2.0 ** -20)
    union = np.union1d(a.cells, b.cells)
    excluded = _near_zero_cells(S, n, lo, h, union, floor)
    ka, kb = ~np.isin(a.cells, excluded), ~np.isin(b.cells, excluded)
    print(f"N={n}: {len(a.cells)} (f32) / {len(b.cells)} (f64) sign-change cells, {len(excluded)} set aside "
          f"(a corner |f64| < {floor:.2e}), {len(np.setxor1d(a.cells, b.cells))} differ", flush=True)
    np.testing.assert_array_equal(a.cells[ka], b.cells[kb])
    np.testing.assert_array_equal(a.cases[ka], b.cases[kb])
    assert len(excluded) <= 2 * 16 * floor / h * len(b.cells)
    # vertices: with |f32 - f64| <= E = 2e-6 at each end (test_fp32_twin_agrees_with_fp64)
    # and f_a, f_b of opposite signs, t = f_a/(f_a - f_b) moves by at most
    # E (|f_a| + |f_b|)/(f_a - f_b)^2 = E/|f_a - f_b| to first order
    common, ia, ib = np.intersect1d(a.edge_ids, b.edge_ids, return_indices=True)
    assert len(common) >= 0.999 * len(b.edge_ids)
    n1 = n + 1
    axis, lower = common % 3, common // 3
    upper = lower + np.where(axis == 0, n1 * n1, np.where(axis == 1, n1, 1))
    ends = [np.stack([mc.lattice_coords_f64(n, lo, h, v) for v in (q // (n1 * n1), (q // n1) % n1, q % n1)], axis=1)
            for q in (lower, upper)]
    gap = np.abs(S.f64(ends[0]) - S.f64(ends[1]))
    dt = np.abs(a.ts[ia] - b.ts[ib])
    print(f"N={n}: {len(common)} vertices, max |t32 - t64| {dt.max():.2e}, "
          f"max |t32 - t64| |f_a - f_b| {(dt * gap).max():.2e}", flush=True)
    assert np.all(dt * gap <= 2e-6 * 1.01)


@pytest.mark.parametrize("scene", ["sphere", "csg"])
def test_shrunk_hop_rule_keeps_every_cell(scene):
    """The bf16 hop rule: a value known only to within eps of f steps
    floor(max(|f| - eps, 0)/h).  It still reaches every cell the surface
    crosses (the mesh equals enumeration's), with at least as many
    evaluations and candidates as the exact rule; a planted sign mistake
    (|f| + eps) skips cells."""
    recs = W.sphere_scene(0.5) if scene == "sphere" else W.csg_scene(2)
    S = sdb.SDB.prims(recs)
    n, lo, h = W.grid(48)
    dense, _ = mc.enumerate_mesh(S, n, lo, h)
    exact = hop.gridhop(S, n, lo, h)
    for eps in (0.3 * h, 1.7 * h):
        r = hop.gridhop(S, n, lo, h, shrink=eps)
        assert _mesh_equal(r.mesh, dense)
        assert np.all(np.isin(dense.cells, r.candidates))
        assert r.hop_evals >= exact.hop_evals and len(r.candidates) >= len(exact.candidates)
    # planted: the margin added instead of subtracted
    cells, _, _ = hop.hop(S, n, lo, h, shrink=-1.7 * h)
    assert not np.all(np.isin(dense.cells, cells))
